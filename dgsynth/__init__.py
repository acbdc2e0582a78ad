"""Seeded synthetic DG-shaped linear systems for the transformed Radau IIA solve.

This module only draws inputs.  It holds none of the solver's arithmetic
(no tableau, no operator, no factorization): it builds a mesh adjacency,
draws the block Jacobian J, the block-diagonal mass matrix M and a right-hand
side, and hands them out as plain NumPy arrays.  Both the HIP path and the
CPU oracle consume exactly these arrays.

Structure follows the paper's block description (Sec. 2.1, "Block structure
of the Jacobian"): T elements, m unknowns per element, J is a T x T block
matrix of dense m x m blocks that is nonzero on the diagonal and where two
elements share a face; M is block diagonal.  The paper's meshes and
Jacobians come from a DG flow solver that is not available, so seeded
synthetic values of the same shape stand in for them:

* mesh: periodic N x N quad grid (4 face neighbours) or periodic N^3 hex grid
  (6 face neighbours); a non-periodic path (tree) and an isolated-element
  mesh exist for special-case tests;
* element numbering: a seeded random permutation, new label of old element
  ``e`` is ``perm[e]``;
* J blocks: off-diagonal blocks N(0,1)/sqrt(m); diagonal blocks
  -(4 I + N(0,1)/sqrt(m));
* M blocks: I + 0.1 R R^T / m with R an m x m matrix of N(0,1) entries;
* right-hand side: N(0,1), stage-major [s][T][m].

Draw order (one ``numpy.random.default_rng(seed)`` stream):
``perm``; then J values for k in range(nJ), block rows in new-label order,
blocks within a row in ascending column order (diagonal included); then M
for elements in new-label order; then the right-hand side.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "grid2d", "grid3d", "path_mesh", "isolated_mesh", "System", "make_system",
    "config_system", "batch_specs", "serve_requests", "CONFIGS",
]


# ----------------------------------------------------------------------------
# meshes (neighbour lists in the mesh's own "old" labels)
# ----------------------------------------------------------------------------

def grid2d(N: int) -> List[List[int]]:
    """Periodic N x N quad grid, 4 face neighbours per element.

    N >= 4 is required: for N <= 3 two neighbours of an element can be
    neighbours of each other (or coincide), which breaks the triangle-free
    condition of the simplified block ILU(0) (Sec. 4.2.1, Alg. 2).
    """
    if N < 4:
        raise ValueError("periodic grid side must be >= 4 (triangle-free mesh)")
    nb = []
    for a in range(N):
        for b in range(N):
            nb.append(sorted({((a + 1) % N) * N + b, ((a - 1) % N) * N + b,
                              a * N + (b + 1) % N, a * N + (b - 1) % N}))
    return nb


def grid3d(N: int) -> List[List[int]]:
    """Periodic N^3 hex grid, 6 face neighbours per element (N >= 4)."""
    if N < 4:
        raise ValueError("periodic grid side must be >= 4 (triangle-free mesh)")
    nb = []
    idx = lambda a, b, c: (a % N) * N * N + (b % N) * N + (c % N)
    for a in range(N):
        for b in range(N):
            for c in range(N):
                nb.append(sorted({idx(a + 1, b, c), idx(a - 1, b, c),
                                  idx(a, b + 1, c), idx(a, b - 1, c),
                                  idx(a, b, c + 1), idx(a, b, c - 1)}))
    return nb


def path_mesh(T: int) -> List[List[int]]:
    """Non-periodic chain of T elements (a tree: block ILU(0) is exact on it
    in natural order)."""
    return [[j for j in (e - 1, e + 1) if 0 <= j < T] for e in range(T)]


def isolated_mesh(T: int) -> List[List[int]]:
    """T elements with no face neighbours (r = 0)."""
    return [[] for _ in range(T)]


# ----------------------------------------------------------------------------
# one system
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class System:
    """One synthetic system.  Arrays are C-contiguous.

    row_ptr : int32 [T+1]          block-row pointers (BSR)
    col_idx : int32 [nnzb]         ascending within a row, diagonal included
    J       : float64 [nJ, nnzb, m, m]   row-major blocks
    M       : float64 [T, m, m]          row-major blocks
    rhs     : float64 [s*T*m]            stage-major [s][T][m]
    perm    : int64 [T]                  new label of old element e
    """
    s: int
    T: int
    m: int
    nJ: int
    dt: float
    row_ptr: np.ndarray
    col_idx: np.ndarray
    J: np.ndarray
    M: np.ndarray
    rhs: np.ndarray
    perm: np.ndarray
    seed: object = None
    name: str = ""

    @property
    def nnzb(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def n(self) -> int:
        return self.T * self.m


def make_system(seed, mesh: Sequence[Sequence[int]], m: int, s: int, dt: float,
                nJ: int = 1, permute: bool = True, name: str = "",
                scale: Optional[float] = None, diag_shift: float = 4.0,
                mass_weight: float = 0.1) -> System:
    """Draw one system on the given mesh (see module docstring for the recipe)."""
    rng = np.random.default_rng(seed)
    T = len(mesh)
    if permute:
        perm = rng.permutation(T)
    else:
        perm = np.arange(T)
    # neighbour sets in new labels
    rows = [None] * T
    for e in range(T):
        i = int(perm[e])
        cols = {i}
        for f in mesh[e]:
            cols.add(int(perm[f]))
        rows[i] = sorted(cols)
    row_ptr = np.zeros(T + 1, dtype=np.int32)
    for i in range(T):
        row_ptr[i + 1] = row_ptr[i] + len(rows[i])
    col_idx = np.fromiter((j for i in range(T) for j in rows[i]), dtype=np.int32,
                          count=int(row_ptr[-1]))
    nnzb = int(row_ptr[-1])
    sc = (1.0 / math.sqrt(m)) if scale is None else scale
    J = rng.standard_normal((nJ, nnzb, m, m))
    J *= sc
    # diagonal blocks: -(4 I + G)
    rowid = np.repeat(np.arange(T, dtype=np.int64), np.diff(row_ptr))
    dpos = np.nonzero(col_idx.astype(np.int64) == rowid)[0]
    eye = np.eye(m)
    for k in range(nJ):
        J[k, dpos] += diag_shift * eye
        J[k, dpos] *= -1.0
    R = rng.standard_normal((T, m, m))
    M = np.matmul(R, R.transpose(0, 2, 1))
    M *= mass_weight / m
    M += eye
    rhs = rng.standard_normal(s * T * m)
    return System(s=s, T=T, m=m, nJ=nJ, dt=float(dt), row_ptr=row_ptr,
                  col_idx=col_idx, J=np.ascontiguousarray(J),
                  M=np.ascontiguousarray(M), rhs=rhs, perm=perm, seed=seed,
                  name=name)


# ----------------------------------------------------------------------------
# the named workloads
# ----------------------------------------------------------------------------

#: Named workloads.  ``mesh`` is (dim, N); m = components * (p+1)^dim.
CONFIGS = {
    # plain method, FP64, tiny (dense LU feasible): s=2, 8x8, p=1, 4 comps
    "cfg0": dict(s=2, dim=2, N=8, m=16, dt=0.1, pc="coupled", rtol=1e-10),
    # plain method on GPU, FP64: s=3, 64x64, p=3, 4 comps
    "cfg1": dict(s=3, dim=2, N=64, m=64, dt=0.1, pc="coupled", rtol=1e-10,
                 dts=(0.01, 0.1, 1.0), pcs=("coupled", "uncoupled_shifted")),
    # precision: s=3, 16^3 hex, p=2, 5 comps
    "cfg2": dict(s=3, dim=3, N=16, m=135, dt=0.5, pc="uncoupled_shifted",
                 rtol=1e-8),
}


def config_system(name: str, instance: int = 0, dt: Optional[float] = None,
                  N: Optional[int] = None, nJ: int = 1) -> System:
    """System of a named workload.  Seeds are 1000*config_index + instance.

    ``N`` overrides the mesh side (same value recipe on a smaller mesh)."""
    cfg = CONFIGS[name]
    idx = int(name[3:])
    NN = cfg["N"] if N is None else N
    mesh = grid2d(NN) if cfg["dim"] == 2 else grid3d(NN)
    return make_system(1000 * idx + instance, mesh, cfg["m"], cfg["s"],
                       cfg["dt"] if dt is None else dt, nJ=nJ,
                       name=f"{name}" + ("" if N is None else f"@N={N}"))


@dataclasses.dataclass
class Spec:
    """Size of one system in a batch or request stream."""
    dim: int
    N: int
    p: int
    comps: int
    s: int
    dt: float
    seed: object

    @property
    def m(self) -> int:
        return self.comps * (self.p + 1) ** self.dim

    @property
    def T(self) -> int:
        return self.N ** self.dim

    def build(self) -> System:
        mesh = grid2d(self.N) if self.dim == 2 else grid3d(self.N)
        return make_system(self.seed, mesh, self.m, self.s, self.dt,
                           name=f"{self.dim}d N={self.N} p={self.p} s={self.s}")


def batch_specs(count: int = 256, seed: int = 3000, Nmin: int = 4, Nmax: int = 32,
                pmax: int = 4) -> List[Spec]:
    """Uneven batch: N ~ U{Nmin..Nmax} periodic 2D grid, p ~ U{1..pmax},
    4 components (m = 4 (p+1)^2), s ~ U{2,3,4}, dt = 10^U(-2, 0)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.integers(Nmin, Nmax + 1))
        p = int(rng.integers(1, pmax + 1))
        s = int(rng.integers(2, 5))
        dt = float(10.0 ** rng.uniform(-2.0, 0.0))
        out.append(Spec(2, N, p, 4, s, dt, (seed, i)))
    return out


def serve_requests(count: int, seed: int = 4000, N2max: int = 64, N3max: int = 16,
                   reuse_frac: float = 0.3):
    """Request stream: 75 % 2D (N ~ U{4..N2max}, p ~ U{1..4}, 4 comps),
    25 % 3D (N ~ U{4..N3max}, p = 2, 5 comps); s ~ U{2,3,4}; a fraction
    ``reuse_frac`` re-uses the operator of an earlier request with a fresh
    right-hand side.  Returns a list of (Spec, reuse_of or None, rhs_seed)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        if out and rng.uniform() < reuse_frac:
            j = int(rng.integers(0, len(out)))
            base = out[j][1] if out[j][1] is not None else j
            out.append((out[base][0], base, (seed, i, 1)))
            continue
        if rng.uniform() < 0.75:
            spec = Spec(2, int(rng.integers(4, N2max + 1)), int(rng.integers(1, 5)), 4,
                        int(rng.integers(2, 5)), float(10.0 ** rng.uniform(-2, 0)),
                        (seed, i))
        else:
            spec = Spec(3, int(rng.integers(4, N3max + 1)), 2, 5,
                        int(rng.integers(2, 5)), float(10.0 ** rng.uniform(-2, 0)),
                        (seed, i))
        out.append((spec, None, (seed, i, 1)))
    return out


def fresh_rhs(seed, s: int, T: int, m: int) -> np.ndarray:
    """A new N(0,1) right-hand side for a re-used operator."""
    return np.random.default_rng(seed).standard_normal(s * T * m)
