"""Seeded synthetic inputs: the model operators and right-hand sides.

This module only builds input data. It holds none of the solver's arithmetic
(no weights, matching, prolongators, Galerkin products, smoothers or Krylov
steps), so both the CPU oracle and the GPU library can be fed from it.

Operators (Section 4, eq. (bench); anisotropic variant of the supplementary
anisotropic-Poisson section):

* ``laplacian7(N)``: the 7-point finite-difference Laplacian on the N^3
  interior grid of the unit cube with homogeneous Dirichlet conditions
  eliminated, scaled so the diagonal is 6 and every off-diagonal is -1.
* ``diffusion7(N, kx, ky, kz)``: the 7-point operator of
  -div(K grad u) with a per-node diagonal coefficient K = diag(kx, ky, kz).
  An interior face takes the harmonic mean 2 k_i k_j / (k_i + k_j) of the
  two node coefficients along its axis; a face on the Dirichlet boundary
  takes the node's own coefficient. a_ij = -face, a_ii = sum of the six
  faces. Constant coefficients reduce this to the usual scaled stencil.

Grid ordering is lexicographic with x fastest: i = x + N (y + N z). CSR rows
hold strictly ascending column indices with the diagonal stored. Index
arrays are int32 and values float64; the matrix is bitwise symmetric.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "Csr",
    "laplacian7",
    "diffusion7",
    "block_log_uniform_eps",
    "csr_matvec",
    "small_case",
    "headline_case",
    "aniso_blocks_case",
    "multi_rhs_case",
    "serving_requests",
    "random_spd_graph",
]


class Csr:
    """A square CSR matrix on the host (int32 indices, float64 values)."""

    __slots__ = ("n", "row_ptr", "col", "val")

    def __init__(self, n, row_ptr, col, val):
        self.n = int(n)
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
        self.col = np.ascontiguousarray(col, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        d[rows, self.col] = self.val
        return d


# Neighbour offsets in ascending column order: -z, -y, -x, self, +x, +y, +z.
_AXES = ("z", "y", "x", None, "x", "y", "z")
_SIGNS = (-1, -1, -1, 0, 1, 1, 1)


def _assemble(N: int, off_vals, diag) -> Csr:
    """Assemble a 7-point CSR from per-direction face values.

    ``off_vals[k]`` is an (n,) array with the off-diagonal value of slot k
    (ignored where the neighbour lies outside the grid), ``diag`` is (n,).
    """
    n = N * N * N
    idx = np.arange(n, dtype=np.int64)
    x = idx % N
    y = (idx // N) % N
    z = idx // (N * N)
    coord = {"x": x, "y": y, "z": z}
    stride = {"x": 1, "y": N, "z": N * N}
    cols = np.empty((n, 7), dtype=np.int64)
    vals = np.empty((n, 7), dtype=np.float64)
    mask = np.empty((n, 7), dtype=bool)
    for k, (ax, sg) in enumerate(zip(_AXES, _SIGNS)):
        if ax is None:
            cols[:, k] = idx
            vals[:, k] = diag
            mask[:, k] = True
            continue
        c = coord[ax]
        ok = (c > 0) if sg < 0 else (c < N - 1)
        cols[:, k] = idx + sg * stride[ax]
        vals[:, k] = off_vals[k]
        mask[:, k] = ok
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask]
    if row_ptr[-1] >= 2**31:
        raise ValueError("matrix too large for int32 row offsets")
    return Csr(n, row_ptr.astype(np.int32), col, val)


def laplacian7(N: int) -> Csr:
    """7-point Dirichlet Laplacian on an N^3 interior grid (diag 6, off -1)."""
    if N < 1:
        raise ValueError("N must be positive")
    n = N * N * N
    minus_one = np.full(n, -1.0)
    off = [minus_one] * 7
    return _assemble(N, off, np.full(n, 6.0))


def diffusion7(N: int, kx, ky, kz) -> Csr:
    """7-point diffusion operator with per-node coefficients (kx, ky, kz).

    Each coefficient is a scalar or an (N^3,) array of positive values.
    """
    n = N * N * N
    k = {
        "x": np.broadcast_to(np.asarray(kx, dtype=np.float64), (n,)).copy(),
        "y": np.broadcast_to(np.asarray(ky, dtype=np.float64), (n,)).copy(),
        "z": np.broadcast_to(np.asarray(kz, dtype=np.float64), (n,)).copy(),
    }
    for a in k.values():
        if np.any(a <= 0) or not np.all(np.isfinite(a)):
            raise ValueError("diffusion coefficients must be positive and finite")
    idx = np.arange(n, dtype=np.int64)
    coord = {"x": idx % N, "y": (idx // N) % N, "z": idx // (N * N)}
    stride = {"x": 1, "y": N, "z": N * N}
    # face[ax][sign] = coefficient of the face between node i and its
    # neighbour in direction (ax, sign); own coefficient on the boundary.
    face = {}
    for ax in ("x", "y", "z"):
        kk = k[ax]
        c = coord[ax]
        # face between i and i + stride (the "+" face of i); computed once per
        # face so both rows hold the identical bits.
        plus = kk.copy()
        inner = c < N - 1
        ki = kk[inner]
        kj = kk[idx[inner] + stride[ax]]
        plus[inner] = (2.0 * ki * kj) / (ki + kj)
        minus = kk.copy()
        has_minus = c > 0
        minus[has_minus] = plus[idx[has_minus] - stride[ax]]
        face[ax] = (minus, plus)
    diag = (
        face["x"][0] + face["x"][1] + face["y"][0] + face["y"][1] + face["z"][0] + face["z"][1]
    )
    off = []
    for ax, sg in zip(_AXES, _SIGNS):
        if ax is None:
            off.append(None)
        else:
            off.append(-(face[ax][0] if sg < 0 else face[ax][1]))
    return _assemble(N, off, diag)


def block_log_uniform_eps(N: int, block: int, rng: np.random.Generator):
    """Per-node (eps_x, eps_y) constant on block^3 sub-cubes.

    Blocks are visited in lexicographic block order (x fastest); for each,
    eps_x then eps_y are drawn as 10**uniform(-3, 0) from ``rng``.
    """
    if N % block:
        raise ValueError("N must be a multiple of the block size")
    nb = N // block
    draws = 10.0 ** rng.uniform(-3.0, 0.0, size=(nb * nb * nb, 2))
    idx = np.arange(N * N * N, dtype=np.int64)
    bx = (idx % N) // block
    by = ((idx // N) % N) // block
    bz = (idx // (N * N)) // block
    b = bx + nb * (by + nb * bz)
    return draws[b, 0], draws[b, 1]


def csr_matvec(A: Csr, x: np.ndarray) -> np.ndarray:
    """y = A x with scipy (input construction only, e.g. b = A u)."""
    return A.to_scipy() @ x


# ---------------------------------------------------------------------------
# Workloads. Each returns a dict of host arrays; nothing here touches a GPU.
# ---------------------------------------------------------------------------

def small_case(N: int = 20, seed: int = 0):
    """Isotropic Poisson on N^3 with b ~ U(-1, 1) from ``seed``; x0 = 0."""
    A = laplacian7(N)
    b = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    return {"A": A, "b": b, "N": N, "rtol": 1e-6}


def headline_case(N: int = 160, seed: int = 1):
    """Isotropic Poisson on N^3 with u ~ U(-1, 1) from ``seed`` and b = A u."""
    A = laplacian7(N)
    u = np.random.default_rng(seed).uniform(-1.0, 1.0, A.n)
    b = csr_matvec(A, u)
    return {"A": A, "b": b, "u": u, "N": N, "rtol": 1e-8}


def aniso_blocks_case(N: int = 256, block: int = 16, seed: int = 2):
    """Anisotropic diffusion with (eps_x, eps_y, 1) per block^3 sub-cube.

    eps drawn log-uniform in [1e-3, 1] per block (eps_x then eps_y, block
    order), then b ~ U(-1, 1) from the same generator.
    """
    rng = np.random.default_rng(seed)
    ex, ey = block_log_uniform_eps(N, block, rng)
    A = diffusion7(N, ex, ey, 1.0)
    b = rng.uniform(-1.0, 1.0, A.n)
    return {"A": A, "b": b, "N": N, "rtol": 1e-8}


def multi_rhs_case(N: int = 128, k: int = 32, seed: int = 3):
    """Isotropic Poisson on N^3 with an (n, k) row-major block of U(-1, 1) RHS."""
    A = laplacian7(N)
    B = np.random.default_rng(seed).uniform(-1.0, 1.0, (A.n, k))
    return {"A": A, "B": np.ascontiguousarray(B), "N": N, "rtol": 1e-8}


def serving_requests(count: int, rate: float, seed: int = 4,
                     sizes=(32, 48, 64, 96, 128, 192), p_aniso=0.5, p_reuse=0.5):
    """A Poisson-process request stream of 7-point diffusion solves.

    Per request, in order: exponential inter-arrival gap (mean 1/rate); a
    reuse coin (with probability ``p_reuse`` and at least one operator
    issued, reuse one drawn uniformly from those issued); otherwise a new
    operator: N uniform in ``sizes``, an anisotropy coin (``p_aniso``) and,
    if anisotropic, constant eps_x, eps_y = 10**U(-3, 0). Every request gets
    a fresh RHS seed. Returns a list of dicts (operators are described, not
    assembled: ``op_id``, ``N``, ``eps``).
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    ops = []
    reqs = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        reuse = rng.uniform() < p_reuse
        if reuse and ops:
            op = ops[int(rng.integers(len(ops)))]
        else:
            N = int(sizes[int(rng.integers(len(sizes)))])
            aniso = rng.uniform() < p_aniso
            eps = (1.0, 1.0)
            if aniso:
                e = 10.0 ** rng.uniform(-3.0, 0.0, size=2)
                eps = (float(e[0]), float(e[1]))
            op = {"op_id": len(ops), "N": N, "eps": eps}
            ops.append(op)
        reqs.append({"req_id": r, "t_arrival": t, "op_id": op["op_id"], "N": op["N"],
                     "eps": op["eps"], "rhs_seed": int(rng.integers(2**31 - 1))})
    return reqs


def request_operator(req) -> Csr:
    """Assemble the operator a serving request refers to."""
    ex, ey = req["eps"]
    if ex == 1.0 and ey == 1.0:
        return laplacian7(req["N"])
    return diffusion7(req["N"], ex, ey, 1.0)


def request_rhs(req) -> np.ndarray:
    n = req["N"] ** 3
    return np.random.default_rng(req["rhs_seed"]).uniform(-1.0, 1.0, n)


def random_spd_graph(n: int, avg_deg: float, seed: int, diag_shift: float = 0.5,
                     hub_degree: int = 0) -> Csr:
    """A random symmetric diagonally dominant (hence s.p.d.) sparse matrix.

    Off-diagonal values are -U(0.1, 1) on a random symmetric pattern; the
    diagonal is the row's absolute off-diagonal sum plus ``diag_shift``.
    ``hub_degree`` > 0 connects vertex 0 to that many others (long rows).
    """
    rng = np.random.default_rng(seed)
    m = int(n * avg_deg / 2)
    i = rng.integers(0, n, m)
    j = rng.integers(0, n, m)
    if hub_degree > 0:
        hub = rng.choice(np.arange(1, n), size=min(hub_degree, n - 1), replace=False)
        i = np.concatenate([i, np.zeros(len(hub), dtype=i.dtype)])
        j = np.concatenate([j, hub])
    keep = i != j
    lo = np.minimum(i[keep], j[keep])
    hi = np.maximum(i[keep], j[keep])
    key = np.unique(lo.astype(np.int64) * n + hi)
    lo = key // n
    hi = key % n
    v = -rng.uniform(0.1, 1.0, len(lo))
    rows = np.concatenate([lo, hi, np.arange(n)])
    cols = np.concatenate([hi, lo, np.arange(n)])
    absum = np.zeros(n)
    np.add.at(absum, lo, -v)
    np.add.at(absum, hi, -v)
    vals = np.concatenate([v, v, absum + diag_shift])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Csr(n, row_ptr, cols, vals)


def constant_diffusion7_arrays(N: int, kx: float, ky: float, kz: float, xp, device=None):
    """7-point operator with constant coefficients, built with array module
    ``xp`` (numpy, or torch with ``device``): off-diagonals -k_d along axis d,
    diagonal 2 (kx + ky + kz) (Dirichlet faces take the node's coefficient).
    Returns (row_ptr int32, col int32, val float64) in the CSR conventions of
    this module. Used by serving clients to build operators where they live.
    """
    n = N * N * N
    if xp.__name__ == "torch":
        import torch

        ar = lambda m: torch.arange(m, dtype=torch.int64, device=device)  # noqa: E731
        full = lambda v: torch.full((n,), v, dtype=torch.float64, device=device)  # noqa: E731
        stack = lambda a: torch.stack(a, dim=1)  # noqa: E731
        cumsum = lambda a: torch.cumsum(a, 0)  # noqa: E731
        zero = torch.zeros(1, dtype=torch.int64, device=device)
    else:
        ar = lambda m: np.arange(m, dtype=np.int64)  # noqa: E731
        full = lambda v: np.full(n, v, dtype=np.float64)  # noqa: E731
        stack = lambda a: np.stack(a, axis=1)  # noqa: E731
        cumsum = lambda a: np.cumsum(a)  # noqa: E731
        zero = np.zeros(1, dtype=np.int64)
    idx = ar(n)
    coord = {"x": idx % N, "y": (idx // N) % N, "z": idx // (N * N)}
    stride = {"x": 1, "y": N, "z": N * N}
    kval = {"x": float(kx), "y": float(ky), "z": float(kz)}
    cols, vals, masks = [], [], []
    for ax, sg in zip(_AXES, _SIGNS):
        if ax is None:
            cols.append(idx)
            vals.append(full(2.0 * (float(kx) + float(ky) + float(kz))))
            masks.append(idx >= 0)
            continue
        c = coord[ax]
        masks.append((c > 0) if sg < 0 else (c < N - 1))
        cols.append(idx + sg * stride[ax])
        vals.append(full(-kval[ax]))
    M = stack(masks)
    col = stack(cols)[M]
    val = stack(vals)[M]
    counts = M.sum(1)
    if xp.__name__ == "torch":
        import torch

        row_ptr = torch.cat([zero, cumsum(counts)]).to(torch.int32)
        return row_ptr.contiguous(), col.to(torch.int32).contiguous(), val.contiguous()
    row_ptr = np.concatenate([zero, cumsum(counts)]).astype(np.int32)
    return row_ptr, col.astype(np.int32), val


def diffusion7_torch(N: int, kx, ky, kz, device):
    """diffusion7 built with torch on ``device`` (same operations, same bits).

    ``kx, ky, kz`` are scalars or (N^3,) float64 tensors/arrays. Returns
    (row_ptr int32, col int32, val float64) tensors in this module's CSR
    conventions.
    """
    import torch

    n = N * N * N

    def coef(v):
        t = torch.as_tensor(v, dtype=torch.float64, device=device)
        return t.expand(n).clone() if t.dim() == 0 else t.clone()

    k = {"x": coef(kx), "y": coef(ky), "z": coef(kz)}
    idx = torch.arange(n, dtype=torch.int64, device=device)
    coord = {"x": idx % N, "y": (idx // N) % N, "z": idx // (N * N)}
    stride = {"x": 1, "y": N, "z": N * N}
    face = {}
    for ax in ("x", "y", "z"):
        kk = k[ax]
        c = coord[ax]
        plus = kk.clone()
        inner = c < N - 1
        ki = kk[inner]
        kj = kk[idx[inner] + stride[ax]]
        plus[inner] = (2.0 * ki * kj) / (ki + kj)
        minus = kk.clone()
        has_minus = c > 0
        minus[has_minus] = plus[idx[has_minus] - stride[ax]]
        face[ax] = (minus, plus)
    diag = (face["x"][0] + face["x"][1] + face["y"][0] + face["y"][1] + face["z"][0]
            + face["z"][1])
    cols, vals, masks = [], [], []
    for ax, sg in zip(_AXES, _SIGNS):
        if ax is None:
            cols.append(idx)
            vals.append(diag)
            masks.append(torch.ones(n, dtype=torch.bool, device=device))
            continue
        c = coord[ax]
        masks.append((c > 0) if sg < 0 else (c < N - 1))
        cols.append(idx + sg * stride[ax])
        vals.append(-(face[ax][0] if sg < 0 else face[ax][1]))
    M = torch.stack(masks, dim=1)
    col = torch.stack(cols, dim=1)[M].to(torch.int32).contiguous()
    val = torch.stack(vals, dim=1)[M].contiguous()
    counts = M.sum(1)
    row_ptr = torch.cat([torch.zeros(1, dtype=torch.int64, device=device),
                         torch.cumsum(counts, 0)]).to(torch.int32).contiguous()
    return row_ptr, col, val


def aniso_blocks_coefficients(N: int = 256, block: int = 16, seed: int = 2):
    """(eps_x, eps_y) per node and the right-hand side of aniso_blocks_case,
    drawn in the same order from the same generator (no operator assembly)."""
    rng = np.random.default_rng(seed)
    ex, ey = block_log_uniform_eps(N, block, rng)
    b = rng.uniform(-1.0, 1.0, N ** 3)
    return ex, ey, b
