"""Seeded synthetic spectrahedra (LMIs) and start points.

This module only draws random matrices; it holds none of the boundary-oracle
arithmetic, so both the HIP path and the CPU reference can take their inputs
from it.

An instance is an LMI F(x) = A0 + sum_i x_i A_i (the paper's eq. (1)) given as
a list of blocks, F(x) = blkdiag_b F_b(x):
  * a DENSE block of size m is an array of shape (n+1, m, m) of symmetric
    matrices A_{b,0..n};
  * a DIAG block of size m is an array of shape (n+1, m) of diagonals, i.e.
    m scalar linear inequalities (a polytope's rows).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np

DENSE = 0
DIAG = 1


@dataclasses.dataclass
class Block:
    kind: int
    A: np.ndarray  # (n+1, m, m) for DENSE, (n+1, m) for DIAG

    @property
    def m(self) -> int:
        return int(self.A.shape[1])


@dataclasses.dataclass
class Instance:
    n: int
    blocks: List[Block]
    name: str = ""

    def flat(self) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
        """(block sizes int32, kinds int32, concatenated float64 coefficients)."""
        sizes = np.array([b.m for b in self.blocks], dtype=np.int32)
        kinds = np.array([b.kind for b in self.blocks], dtype=np.int32)
        A = np.concatenate([np.ascontiguousarray(b.A, dtype=np.float64).ravel() for b in self.blocks])
        return sizes, kinds, A

    def dense_m(self) -> int:
        return sum(b.m for b in self.blocks if b.kind == DENSE)

    def dense_matrix(self) -> np.ndarray:
        """The same LMI as one dense block-diagonal (n+1, M, M) stack."""
        M = sum(b.m for b in self.blocks)
        out = np.zeros((self.n + 1, M, M))
        o = 0
        for b in self.blocks:
            if b.kind == DENSE:
                out[:, o:o + b.m, o:o + b.m] = b.A
            else:
                idx = np.arange(o, o + b.m)
                out[:, idx, idx] = b.A
            o += b.m
        return out


def _sym_gaussian(rng: np.random.Generator, n: int, m: int, scale: float) -> np.ndarray:
    G = rng.standard_normal((n, m, m))
    return (G + G.transpose(0, 2, 1)) / (2.0 * scale)


def box_block(n: int, half_width: float = 10.0) -> Block:
    """DIAG block of size 2n: half_width - x_i >= 0 and half_width + x_i >= 0."""
    A = np.zeros((n + 1, 2 * n))
    A[0, :] = half_width
    for i in range(n):
        A[i + 1, i] = -1.0
        A[i + 1, n + i] = 1.0
    return Block(DIAG, A)


def gbase(n: int, m: int, seed: int, scale: float | None = None, box: bool = True) -> Instance:
    """Dense block A0 = I_m, A_i = (G_i + G_i^T) / (2 s), G_i entries N(0,1),
    with s = sqrt(m) unless given, plus the box |x_i| <= 10 as a DIAG block."""
    rng = np.random.default_rng(seed)
    s = math.sqrt(m) if scale is None else scale
    A = np.empty((n + 1, m, m))
    A[0] = np.eye(m)
    A[1:] = _sym_gaussian(rng, n, m, s)
    blocks = [Block(DENSE, A)]
    if box:
        blocks.append(box_block(n))
    return Instance(n, blocks, name=f"gbase-n{n}-m{m}-s{seed}")


def paper_random(n: int, m: int, seed: int) -> Instance:
    """Random spectrahedron of the paper's experiments (Section 4): A0 = Z Z^T + I
    with Z uniform on [0,1]; A_i = blkdiag(Qt, -Qt), Qt = Q + Q^T with Q uniform
    on [-1,1]^{m/2 x m/2}."""
    if m % 2:
        raise ValueError("m must be even")
    rng = np.random.default_rng(seed)
    Z = rng.uniform(0.0, 1.0, (m, m))
    A = np.zeros((n + 1, m, m))
    A[0] = Z @ Z.T + np.eye(m)
    h = m // 2
    for i in range(n):
        Q = rng.uniform(-1.0, 1.0, (h, h))
        Qt = Q + Q.T
        A[i + 1, :h, :h] = Qt
        A[i + 1, h:, h:] = -Qt
    return Instance(n, [Block(DENSE, A)], name=f"paper-n{n}-m{m}-s{seed}")


def arrow_ball(n: int, radius: float = 1.0) -> Instance:
    """F(x) = [[r, x^T], [x, r I]]: PSD iff |x| <= r (Schur complement); the
    ball of radius r."""
    m = n + 1
    A = np.zeros((n + 1, m, m))
    A[0] = radius * np.eye(m)
    for i in range(n):
        A[i + 1, 0, i + 1] = 1.0
        A[i + 1, i + 1, 0] = 1.0
    return Instance(n, [Block(DENSE, A)], name=f"ball-n{n}")


def polytope(Amat: np.ndarray, b: np.ndarray) -> Instance:
    """{x : Amat x <= b} as one DIAG block: F_jj(x) = b_j - (Amat x)_j."""
    rows, n = Amat.shape
    A = np.zeros((n + 1, rows))
    A[0] = b
    A[1:] = -Amat.T
    return Instance(n, [Block(DIAG, A)], name=f"polytope-{rows}x{n}")


def box(n: int, half_width: float = 1.0) -> Instance:
    return Instance(n, [box_block(n, half_width)], name=f"box-n{n}")


def box_as_dense(n: int, half_width: float = 1.0) -> Instance:
    """The same box written as a dense block with diagonal A_i."""
    bl = box_block(n, half_width)
    m = 2 * n
    A = np.zeros((n + 1, m, m))
    for i in range(n + 1):
        A[i] = np.diag(bl.A[i])
    return Instance(n, [Block(DENSE, A)], name=f"densebox-n{n}")


def simplex(n: int, centered: bool = True) -> Instance:
    """The standard simplex {y >= 0, sum y <= 1} (volume 1/n!), translated by
    its centroid when `centered` so that the origin is interior."""
    c = 1.0 / (n + 1) if centered else 0.0
    Amat = np.vstack([-np.eye(n), np.ones((1, n))])
    b = np.concatenate([np.full(n, c), [1.0 - n * c]])
    return polytope(Amat, b)


def elliptope3() -> Instance:
    """3x3 correlation matrices [[1,x1,x2],[x1,1,x3],[x2,x3,1]] >= 0; volume pi^2/2."""
    A = np.zeros((4, 3, 3))
    A[0] = np.eye(3)
    for i, (r, c) in enumerate([(0, 1), (0, 2), (1, 2)]):
        A[i + 1, r, c] = A[i + 1, c, r] = 1.0
    return Instance(3, [Block(DENSE, A)], name="elliptope3")


def paper_example_2d() -> Instance:
    """The 2-D example of Section 2 with the matrices of Appendix B (rounded
    to one decimal in the paper).  The generator of Section 4 makes
    A_i = blkdiag(Qt, -Qt); the printed lower blocks repeat +Qt and row 1 of A1
    lacks its last entry: read as -Qt and 0."""
    A0 = np.array([
        [16.7, 3.7, 12.3, 8.7, 5.1, 10.4],
        [3.7, 9.4, 2.3, 4.0, -2.3, -1.0],
        [12.3, 2.3, 26.8, 18.7, 7.1, 16.7],
        [8.7, 4.0, 18.7, 20.0, 3.7, 12.3],
        [5.1, -2.3, 7.1, 3.7, 6.1, 5.4],
        [10.4, -1.0, 16.7, 12.3, 5.4, 18.7]])
    Q1 = np.array([[0.5, -0.4, 2.7], [-0.4, 1.4, -0.2], [2.7, -0.2, 1.7]])
    Q2 = np.array([[2.6, -0.1, 3.0], [-0.1, 1.0, -0.1], [3.0, -0.1, -1.0]])
    A = np.zeros((3, 6, 6))
    A[0] = A0
    for i, Q in enumerate([Q1, Q2]):
        A[i + 1, :3, :3] = Q
        A[i + 1, 3:, 3:] = -Q
    return Instance(2, [Block(DENSE, A)], name="paper-example-2d")


def congruent(inst: Instance, seed: int) -> Instance:
    """Q^T A_i Q for a random orthogonal Q on every dense block (same set)."""
    rng = np.random.default_rng(seed)
    out = []
    for b in inst.blocks:
        if b.kind == DENSE:
            Q, _ = np.linalg.qr(rng.standard_normal((b.m, b.m)))
            out.append(Block(DENSE, np.einsum("ji,njk,kl->nil", Q, b.A, Q)))
        else:
            out.append(Block(DIAG, b.A.copy()))
    return Instance(inst.n, out, name=inst.name + "-congruent")


def random_directions(rng: np.random.Generator, batch: int, n: int) -> np.ndarray:
    g = rng.standard_normal((batch, n))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


def interior_points(inst: Instance, rng: np.random.Generator, batch: int, frac: np.ndarray | float,
                    t_plus_fn) -> np.ndarray:
    """Points a fraction `frac` of the way from 0 to the boundary along random
    directions; t_plus_fn(x, v) gives the boundary distance (any oracle)."""
    v = random_directions(rng, batch, inst.n)
    x0 = np.zeros((batch, inst.n))
    tp = t_plus_fn(x0, v)
    f = np.broadcast_to(np.asarray(frac, dtype=np.float64), (batch,))
    return x0 + (f * tp)[:, None] * v


def objective(n: int, seed: int) -> np.ndarray:
    """A seeded unit objective vector c for min <c, x> over S."""
    c = np.random.default_rng(seed).standard_normal(n)
    return c / np.linalg.norm(c)


def sdp_family(sizes=(30, 40, 50, 60), per_size: int = 10):
    """The optimisation workload of the paper's annealing table: per size n,
    `per_size` spectrahedra S-n-n of its generator with seeded objectives;
    entries (n, instance seed, objective seed)."""
    return [(n, 30000 + 100 * n + k, 31000 + 100 * n + k) for n in sizes for k in range(per_size)]


def uneven_family(count: int, seed: int, lo: int = 20, hi: int = 200, balls: int = 16):
    """`count` instances with n and m log-uniform in [lo, hi]; the first
    `balls` are arrow-LMI unit balls of random n (known volume)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        n = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        m = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        if k < balls:
            out.append(arrow_ball(n))
        else:
            out.append(gbase(n, m, seed=int(rng.integers(1 << 31))))
    return out
