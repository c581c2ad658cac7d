"""Seeded synthetic workloads for the DPG local solve.

This module only builds inputs: structured hexahedral meshes (perturbed or
curved), per-cell materials, polynomial degrees, boundary tags and the port
description.  It contains none of the method's arithmetic and is the one
module shared by the oracle-based tests and the GPU path.

Meshes mimic the paper's set-ups (§4.1 waveguide, App. C tables): walls
x-, x+, y-, y+ are perfect conductors, z- is the TE10 port (Robin with mode
data), z+ is an impedance outlet (Robin with g = 0).  Vertex v(i,j,k) of a cell
is stored at position 4k+2j+i of its connectivity row.

Materials are given in the paper's sign convention (time factor e^{-i w t},
lossy => Im(eps) > 0): a quoted permittivity eps'(1 - i tan d) becomes
eps'(1 + i tan d).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

SEED_BASE = 2609031550
C0 = 299_792_458.0

FACE_INTERIOR, FACE_PEC, FACE_PORT, FACE_ROBIN0 = 0, 1, 2, 3


@dataclass
class Workload:
    name: str
    vertices: np.ndarray          # (nv, 3) float64, metres (= non-dimensional, L = 1 m)
    cells: np.ndarray             # (nc, 8) int64
    eps: np.ndarray               # (nc,) complex128
    mu: np.ndarray                # (nc,) complex128
    degree: np.ndarray            # (nc,) int8
    face_kind: np.ndarray         # (nc, 6) int8
    zinv: np.ndarray              # (nc, 6) complex128, Robin admittance per face
    dp: int
    freq_hz: float
    port: dict                    # a, b, m, n, eps, mu of the feed guide
    shape: tuple = ()
    meta: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    def cell_vertices(self, c: int) -> np.ndarray:
        return self.vertices[self.cells[c]]

    def subset(self, idx) -> "Workload":
        idx = np.asarray(idx, dtype=np.int64)
        return Workload(self.name + f"[{len(idx)}]", self.vertices, self.cells[idx], self.eps[idx],
                        self.mu[idx], self.degree[idx], self.face_kind[idx], self.zinv[idx],
                        self.dp, self.freq_hz, dict(self.port), self.shape, dict(self.meta))


def port_admittance(a: float, b: float, m: int, n: int, freq_hz: float,
                    eps: complex = 1.0, mu: complex = 1.0) -> complex:
    """k_x3 / (omega mu) of the TE_mn mode (data for the Robin faces)."""
    om = 2.0 * math.pi * freq_hz / C0
    kc2 = (m * math.pi / a) ** 2 + (n * math.pi / b) ** 2
    k3 = np.sqrt(complex(om * om * eps * mu - kc2))
    return complex(k3 / (om * mu))


def box_mesh(nx, ny, nz, lx, ly, lz, perturb=0.0, rng=None, curve=None):
    """Structured nx x ny x nz hex mesh of [0,lx]x[0,ly]x[0,lz].
    perturb: each vertex coordinate moves by U[-perturb*h_d, +perturb*h_d]
    along every axis d in which the vertex is not on a boundary plane (so the
    box walls stay planar and corners stay fixed).
    curve: optional callable (nv,3) -> (nv,3) applied after perturbation."""
    xs = np.linspace(0.0, lx, nx + 1)
    ys = np.linspace(0.0, ly, ny + 1)
    zs = np.linspace(0.0, lz, nz + 1)
    K, J, I = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing='ij')
    I, J, K = I.ravel(), J.ravel(), K.ravel()
    V = np.stack([xs[I], ys[J], zs[K]], axis=1)
    if perturb > 0.0:
        h = np.array([lx / nx, ly / ny, lz / nz])
        d = rng.uniform(-perturb, perturb, size=V.shape) * h[None, :]
        interior = np.stack([(I > 0) & (I < nx), (J > 0) & (J < ny), (K > 0) & (K < nz)], axis=1)
        V = V + d * interior
    if curve is not None:
        V = curve(V)

    def vid(i, j, k):
        return i + (nx + 1) * (j + (ny + 1) * k)

    ck, cj, ci = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing='ij')
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    cells = np.stack([vid(ci + a, cj + b, ck + c) for c in (0, 1) for b in (0, 1) for a in (0, 1)],
                     axis=1).astype(np.int64)
    fk = np.zeros((cells.shape[0], 6), dtype=np.int8)
    fk[ci == 0, 0] = FACE_PEC
    fk[ci == nx - 1, 1] = FACE_PEC
    fk[cj == 0, 2] = FACE_PEC
    fk[cj == ny - 1, 3] = FACE_PEC
    fk[ck == 0, 4] = FACE_PORT
    fk[ck == nz - 1, 5] = FACE_ROBIN0
    return V, cells, fk, (ci, cj, ck)


def _robin_admittance(fk, y):
    z = np.zeros(fk.shape, dtype=np.complex128)
    z[(fk == FACE_PORT) | (fk == FACE_ROBIN0)] = y
    return z


def waveguide_te10(n: int, p: int, a: float = 0.25, b: float = 0.25, length: float = 1.0,
                   freq_hz: float = 2.45e9) -> Workload:
    """The §4.1 verification guide: a x b x length (0.25 x 0.25 x 1 m), vacuum,
    n x n x 4n uniform hexes of degree p, dp = 1, PEC walls, TE10 port at
    x3 = 0 and the matched impedance outlet at x3 = length."""
    V, cells, fk, _ = box_mesh(n, n, 4 * n, a, b, length)
    nc = cells.shape[0]
    y = port_admittance(a, b, 1, 0, freq_hz)
    return Workload(f"te10_{n}x{n}x{4 * n}_p{p}", V, cells, np.ones(nc, np.complex128), np.ones(nc, np.complex128),
                    np.full(nc, p, np.int8), fk, _robin_admittance(fk, y), 1, freq_hz,
                    dict(a=a, b=b, m=1, n=0, eps=1.0, mu=1.0), (n, n, 4 * n))


def config1() -> Workload:
    """2x2x2 affine mesh of a 0.1 m cube, p=1, dp=1, 2.45 GHz; eps = 1 except
    the cell at the port corner, eps = 4 - 0.5i quoted => 4 + 0.5i here."""
    V, cells, fk, (ci, cj, ck) = box_mesh(2, 2, 2, 0.1, 0.1, 0.1)
    nc = cells.shape[0]
    eps = np.ones(nc, dtype=np.complex128)
    eps[0] = 4.0 + 0.5j
    f = 2.45e9
    port = dict(a=0.1, b=0.1, m=1, n=0, eps=1.0, mu=1.0)
    y = port_admittance(0.1, 0.1, 1, 0, f)
    return Workload("c1_cube_2x2x2_p1", V, cells, eps, np.ones(nc, np.complex128),
                    np.full(nc, 1, np.int8), fk, _robin_admittance(fk, y), 1, f, port, (2, 2, 2))


def config2(nx=16, ny=8, nz=40) -> Workload:
    """WR340-like box 86.36 x 43.18 x 200 mm, 16x8x40 = 5120 hexes, vertices
    perturbed by +-10% of h, p=2, dp=1, eps' ~ U[1,10], tan d ~ U[0,0.3]."""
    rng = np.random.default_rng(SEED_BASE + 2)
    a, b, lz = 0.08636, 0.04318, 0.200
    V, cells, fk, _ = box_mesh(nx, ny, nz, a, b, lz, 0.1, rng)
    nc = cells.shape[0]
    er = rng.uniform(1.0, 10.0, nc)
    td = rng.uniform(0.0, 0.3, nc)
    f = 2.45e9
    port = dict(a=a, b=b, m=1, n=0, eps=1.0, mu=1.0)
    y = port_admittance(a, b, 1, 0, f)
    return Workload(f"c2_wr340_{nx}x{ny}x{nz}_p2", V, cells, er * (1.0 + 1j * td),
                    np.ones(nc, np.complex128), np.full(nc, 2, np.int8), fk,
                    _robin_admittance(fk, y), 1, f, port, (nx, ny, nz))


def config3(nx=25, ny=25, nz=32) -> Workload:
    """0.2 m box, 25x25x32 = 20000 perturbed hexes, p ~ {1,2,3,4} with
    probabilities {0.4,0.3,0.2,0.1}, dp=1; eps = 1 with a seeded 1/8 of the
    cells at 4 + 0.5i."""
    rng = np.random.default_rng(SEED_BASE + 3)
    L = 0.2
    V, cells, fk, _ = box_mesh(nx, ny, nz, L, L, L, 0.1, rng)
    nc = cells.shape[0]
    deg = rng.choice(np.array([1, 2, 3, 4], np.int8), size=nc, p=[0.4, 0.3, 0.2, 0.1])
    eps = np.ones(nc, np.complex128)
    eps[rng.permutation(nc)[: nc // 8]] = 4.0 + 0.5j
    f = 2.45e9
    port = dict(a=L, b=L, m=1, n=0, eps=1.0, mu=1.0)
    y = port_admittance(L, L, 1, 0, f)
    return Workload(f"c3_mixed_p_{nx}x{ny}x{nz}", V, cells, eps, np.ones(nc, np.complex128),
                    deg.astype(np.int8), fk, _robin_admittance(fk, y), 1, f, port, (nx, ny, nz))


def config4(n=16) -> Workload:
    """0.2 m box, 16^3 = 4096 perturbed hexes, p=4, dp=2, eps' ~ U[1,80],
    tan d ~ U[0,0.5], a seeded 1% of hot-spot cells with tan d = 1."""
    rng = np.random.default_rng(SEED_BASE + 4)
    L = 0.2
    V, cells, fk, _ = box_mesh(n, n, n, L, L, L, 0.1, rng)
    nc = cells.shape[0]
    er = rng.uniform(1.0, 80.0, nc)
    td = rng.uniform(0.0, 0.5, nc)
    td[rng.permutation(nc)[: max(1, nc // 100)]] = 1.0
    f = 2.45e9
    port = dict(a=L, b=L, m=1, n=0, eps=1.0, mu=1.0)
    y = port_admittance(L, L, 1, 0, f)
    return Workload(f"c4_highorder_{n}^3_p4dp2", V, cells, er * (1.0 + 1j * td),
                    np.ones(nc, np.complex128), np.full(nc, 4, np.int8), fk,
                    _robin_admittance(fk, y), 2, f, port, (n, n, n))


def smooth_field(rng, n_modes=16, kmax=6 * math.pi):
    """Seeded smooth random field of unit variance: a sum of n_modes cosines
    with wave vectors |k| <= kmax."""
    ks = []
    while len(ks) < n_modes:
        k = rng.uniform(-kmax, kmax, 3)
        if np.linalg.norm(k) <= kmax:
            ks.append(k)
    ks = np.array(ks)
    ph = rng.uniform(0, 2 * math.pi, n_modes)
    amp = math.sqrt(2.0 / n_modes)

    def g(x):
        return amp * np.cos(x @ ks.T + ph[None, :]).sum(axis=1)
    return g


def config5(n=64) -> Workload:
    """[0,1]^3 m, 64^3 = 262144 hexes, vertices mapped x <- x + 0.05 sin(2 pi y)
    sin(2 pi z), p in {2,3} 50/50, dp=1, eps = 3 + 2 tanh(g(x_c)) + 0.3i with a
    smooth random field g evaluated at the cell centroid."""
    rng = np.random.default_rng(SEED_BASE + 5)

    def curve(V):
        V = V.copy()
        V[:, 0] += 0.05 * np.sin(2 * math.pi * V[:, 1]) * np.sin(2 * math.pi * V[:, 2])
        return V

    V, cells, fk, _ = box_mesh(n, n, n, 1.0, 1.0, 1.0, 0.0, None, curve)
    nc = cells.shape[0]
    deg = np.where(rng.uniform(size=nc) < 0.5, 2, 3).astype(np.int8)
    g = smooth_field(rng)
    cen = V[cells].mean(axis=1)
    eps = 3.0 + 2.0 * np.tanh(g(cen)) + 0.3j
    f = 2.45e9
    port = dict(a=1.0, b=1.0, m=1, n=0, eps=1.0, mu=1.0)
    y = port_admittance(1.0, 1.0, 1, 0, f)
    return Workload(f"c5_curved_{n}^3_p23", V, cells, eps.astype(np.complex128),
                    np.ones(nc, np.complex128), deg, fk, _robin_admittance(fk, y), 1, f, port, (n, n, n))


CONFIGS = {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}


def local_dims(p: int, dp: int):
    """(n_test, n_interior, n_trace) = (6 s (s+1)^2, 6 (p+1)^3, 24 (p+1)^2), s = p+dp+1."""
    s = p + dp + 1
    return 6 * s * (s + 1) ** 2, 6 * (p + 1) ** 3, 24 * (p + 1) ** 2


def random_coefficients(w: Workload, seed: int = 7):
    """Seeded complex trial+trace coefficients x_e for every cell, packed at the
    per-cell offsets of the solution layout (k_c = n_interior + n_trace)."""
    rng = np.random.default_rng(SEED_BASE + 100 + seed)
    ks = np.array([sum(local_dims(int(p), w.dp)[1:]) for p in w.degree], np.int64)
    off = np.concatenate([[0], np.cumsum(ks)])
    x = rng.standard_normal(off[-1]) + 1j * rng.standard_normal(off[-1])
    return x.astype(np.complex128), off
