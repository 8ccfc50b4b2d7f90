"""Seeded synthetic inputs for the FEAST hot path.

The paper's matrices (a 2D FEM Kohn-Sham model of a (13,0) carbon nanotube,
Sec. IV.A, and a (5,5) nanotube band-structure family, Sec. IV.C) are not
available, so these block-tridiagonal pencils stand in for them.  They have the
structure of nanowire / nanotube Hamiltonians: a chain of ``nc`` cells of
``b`` orbitals, A real symmetric, B symmetric positive definite, nearest-cell
coupling only (Sec. III.A: A real symmetric, B s.p.d.).

This module only draws numbers.  It holds none of the method's arithmetic, so
both the CPU oracle tests and the GPU path may use it.  Search intervals are
not computed here: they are stored in ``tests/golden/intervals.json`` by a
script that calls only the oracle.

Storage convention shared by every entry point:
  diag[nc][b][b]   diagonal blocks (row-major, symmetric)
  up[nc-1][b][b]   coupling block (i, i+1); the block (i+1, i) is its transpose.
"""
from __future__ import annotations

import dataclasses
import json
import os

import numpy as np

_GOLDEN = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "tests", "golden")


@dataclasses.dataclass
class Pencil:
    """A real symmetric / s.p.d. block-tridiagonal pencil (A, B)."""
    Ad: np.ndarray
    Au: np.ndarray
    Bd: np.ndarray
    Bu: np.ndarray

    @property
    def nc(self) -> int:
        return self.Ad.shape[0]

    @property
    def b(self) -> int:
        return self.Ad.shape[1]

    @property
    def n(self) -> int:
        return self.nc * self.b


def _sym_uniform(rng, nc, b, lo, hi):
    """Symmetric blocks: draw a full block ~U[lo,hi], keep the upper triangle, mirror."""
    m = rng.uniform(lo, hi, size=(nc, b, b))
    up = np.triu(m)
    return up + np.transpose(np.triu(m, 1), (0, 2, 1))


def dense_random_pencil(nc: int, b: int, seed: int, coupling: float = 0.3,
                        b_scale: float = 0.05) -> Pencil:
    """Config-0 recipe: D_i = sym(U[-1,1]); C_i ~ U[-c,c] full, nonsymmetric;
    B = I + b_scale * S with S drawn by the same recipe from an independent stream."""
    sa, sb = np.random.SeedSequence(seed).spawn(2)
    ra, rb = np.random.default_rng(sa), np.random.default_rng(sb)
    Ad = _sym_uniform(ra, nc, b, -1.0, 1.0)
    Au = ra.uniform(-coupling, coupling, size=(max(nc - 1, 0), b, b))
    Sd = _sym_uniform(rb, nc, b, -1.0, 1.0)
    Su = rb.uniform(-coupling, coupling, size=(max(nc - 1, 0), b, b))
    eye = np.eye(b)[None, :, :]
    return Pencil(Ad, Au, eye + b_scale * Sd, b_scale * Su)


def _sparse_hopping(rng, nc, b, per_row):
    """Per cell: each row picks ``per_row`` distinct columns != row with N(0,1)
    values; the block is mirrored (W + W^T), about 2*per_row nonzeros a row."""
    keys = rng.random((nc, b, b))
    idx = np.arange(b)
    keys[:, idx, idx] = np.inf
    cols = np.argsort(keys, axis=2)[:, :, :per_row]
    vals = rng.standard_normal((nc, b, per_row))
    W = np.zeros((nc, b, b))
    cell = np.arange(nc)[:, None, None]
    row = idx[None, :, None]
    W[cell, row, cols] = vals
    return W + np.transpose(W, (0, 2, 1))


def _sparse_coupling(rng, b, per_row, sigma):
    """One coupling block: ``per_row`` random columns a row, values N(0, sigma^2)."""
    keys = rng.random((b, b))
    cols = np.argsort(keys, axis=1)[:, :per_row]
    T = np.zeros((b, b))
    T[np.arange(b)[:, None], cols] = sigma * rng.standard_normal((b, per_row))
    return T


def onsite_potential(amplitudes: np.ndarray, nc: int) -> np.ndarray:
    """Smooth onsite field V(s_i) = sum_k a_k sin(k pi s_i), s_i = (i + 1/2)/nc."""
    s = (np.arange(nc) + 0.5) / nc
    k = np.arange(1, len(amplitudes) + 1)
    return np.sin(np.pi * np.outer(s, k)) @ amplitudes


def chain_pencil(nc: int, b: int, seed: int, amplitudes: np.ndarray | None = None,
                 family_seed: int | None = None) -> Pencil:
    """Config-1 recipe (tight-binding-like chain).

    A: per-cell sparse symmetric hopping (4 draws a row, mirrored) plus a smooth
    onsite potential from 16 Fourier modes; one coupling block T for every cell
    (8 columns a row, N(0, 0.3^2)).  B = I + 0.05 S, S by the same recipe
    without the potential, from an independent stream.

    ``family_seed`` fixes hopping and S for a Hamiltonian family (config 4);
    ``amplitudes`` then selects the member.  Without them the amplitudes are
    one fixed draw from the matrix seed.
    """
    base = family_seed if family_seed is not None else seed
    sa, sb, sv = np.random.SeedSequence(base).spawn(3)
    ra, rb, rv = (np.random.default_rng(s) for s in (sa, sb, sv))
    H = _sparse_hopping(ra, nc, b, 4)
    T = _sparse_coupling(ra, b, 8, 0.3)
    if amplitudes is None:
        amplitudes = 0.5 * rv.standard_normal(16)
    V = onsite_potential(np.asarray(amplitudes, dtype=np.float64), nc)
    Ad = H + V[:, None, None] * np.eye(b)[None]
    Au = np.broadcast_to(T, (max(nc - 1, 0), b, b)).copy()
    S = _sparse_hopping(rb, nc, b, 4)
    TS = _sparse_coupling(rb, b, 8, 0.3)
    Bd = np.eye(b)[None] + 0.05 * S
    Bu = np.broadcast_to(0.05 * TS, (max(nc - 1, 0), b, b)).copy()
    return Pencil(Ad, Au, Bd, Bu)


@dataclasses.dataclass
class HermitianPencil:
    """A complex Hermitian A and a real s.p.d. B in block-tridiagonal storage:
    Ad[nc][b][b] Hermitian, Au[nc-1][b][b] complex with block (i+1, i) =
    Au[i]^H; Bd, Bu real as in Pencil."""
    Ad: np.ndarray
    Au: np.ndarray
    Bd: np.ndarray
    Bu: np.ndarray

    @property
    def nc(self) -> int:
        return self.Ad.shape[0]

    @property
    def b(self) -> int:
        return self.Ad.shape[1]

    @property
    def n(self) -> int:
        return self.nc * self.b


def hermitian_pencil(nc: int, b: int, seed: int, coupling: float = 0.3,
                     phase: float = 0.4, b_scale: float = 0.05) -> HermitianPencil:
    """Complex Hermitian variant of the dense-coupling chain: diagonal blocks
    sym(U[-1,1]) + i phase * antisym(U[-1,1]); couplings U[-c,c] times unit
    phases exp(i phase U[-pi,pi]) (a Peierls-like factor on every hopping);
    B = I + b_scale S, real s.p.d., by the recipe of dense_random_pencil."""
    sa, sb = np.random.SeedSequence(seed).spawn(2)
    ra, rb = np.random.default_rng(sa), np.random.default_rng(sb)
    Dr = _sym_uniform(ra, nc, b, -1.0, 1.0)
    K = ra.uniform(-1.0, 1.0, size=(nc, b, b))
    Di = phase * (K - np.transpose(K, (0, 2, 1))) / 2.0
    Ad = Dr + 1j * Di
    mag = ra.uniform(-coupling, coupling, size=(max(nc - 1, 0), b, b))
    ph = np.exp(1j * phase * ra.uniform(-np.pi, np.pi, size=(max(nc - 1, 0), b, b)))
    Au = mag * ph
    Sd = _sym_uniform(rb, nc, b, -1.0, 1.0)
    Su = rb.uniform(-coupling, coupling, size=(max(nc - 1, 0), b, b))
    eye = np.eye(b)[None, :, :]
    return HermitianPencil(Ad, Au, eye + b_scale * Sd, b_scale * Su)


def hermitian_chain_pencil(nc: int, b: int, seed: int, phase: float = 1.0) -> HermitianPencil:
    """Complex Hermitian variant of the config-1 recipe (a magnetic field on
    the chain): chain_pencil(nc, b, seed) with every hopping entry multiplied
    by a unit phase exp(i phase U[-pi, pi]), antisymmetric inside a diagonal
    block (so that it stays Hermitian) and drawn per cell for the couplings;
    the phases come from a stream of their own, B is the real recipe's."""
    q = chain_pencil(nc, b, seed)
    rp = np.random.default_rng(np.random.SeedSequence(seed).spawn(4)[3])
    th = rp.uniform(-np.pi, np.pi, size=(nc, b, b))
    th = phase * np.triu(th, 1)
    th = th - np.transpose(th, (0, 2, 1))
    Ad = q.Ad * np.exp(1j * th)
    ps = phase * rp.uniform(-np.pi, np.pi, size=(max(nc - 1, 0), b, b))
    Au = q.Au * np.exp(1j * ps)
    return HermitianPencil(Ad, Au, q.Bd, q.Bu)


def random_complex_subspace(n: int, m0: int, seed: int) -> np.ndarray:
    """Complex start block: real and imaginary parts N(0, 1/2) (unit variance)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, m0)) + 1j * rng.standard_normal((n, m0))) / np.sqrt(2.0)


def random_subspace(n: int, m0: int, seed: int) -> np.ndarray:
    """Initial guess Y ~ N(0,1), shape [n][m0] (Fig. 2 step 1: random vectors)."""
    return np.random.default_rng(seed).standard_normal((n, m0))


# --------------------------------------------------------------------------
# Named workloads.  Sizes follow the block-tridiagonal stand-ins for the
# paper's experiments: the small dense-coupling chain (nc=20, b=40), the
# tight-binding chain at full size (nc=2000, b=64, n=128000, M0=128, Ne=8),
# and scaled copies of the latter used by the parity tests.
# --------------------------------------------------------------------------
WORKLOADS = {
    "chain800": dict(kind="dense", nc=20, b=40, M0=30, Ne=8, mseed=1000, yseed=2000,
                     n_eig=20, k0=200),
    "tb128k": dict(kind="chain", nc=2000, b=64, M0=128, Ne=8, mseed=1001, yseed=2001,
                   n_eig=80, k0=32000),
    "tb6400": dict(kind="chain", nc=100, b=64, M0=128, Ne=8, mseed=1001, yseed=2001,
                   n_eig=80, k0=1600),
    "tb32k": dict(kind="chain", nc=500, b=64, M0=64, Ne=8, mseed=4000, yseed=2004,
                  n_eig=38, k0=8000),
    # Hamiltonian family of the learned warm start: the tb32k shape with
    # hopping, coupling and S fixed by the family seed; the interval is the
    # one of the member with a zero onsite potential (38 eigenvalues from
    # index n/4); other members hold 36-50 eigenvalues in it.
    "fam32k": dict(kind="family", nc=500, b=64, M0=64, Ne=8, mseed=4000, yseed=2005,
                   n_eig=38, k0=8000),
    # a small member of the same recipe for the GPU test of the warm start
    "fam1920": dict(kind="family", nc=60, b=32, M0=32, Ne=8, mseed=4000, yseed=2006,
                    n_eig=19, k0=480),
    # Hermitian variant (eq. 12): the tb32k shape of the chain recipe with a
    # phase on every hopping (hermitian_chain_pencil); complex start block
    "htb32k": dict(kind="hchain", nc=500, b=64, M0=64, Ne=8, mseed=1003, yseed=2007,
                   n_eig=38, k0=8000),
}

# Members of the family: s < FAMILY_TRAIN are training members, the next
# FAMILY_TEST held out.  Member s has onsite amplitudes
# a_s = 0.5 * N(0, I_16) drawn from default_rng(FAMILY_SEED + s).
FAMILY_SEED = 4000
FAMILY_MODES = 16
FAMILY_SIGMA = 0.5
FAMILY_TRAIN = 10000
FAMILY_TEST = 1000


def family_amplitudes(s: int) -> np.ndarray:
    return FAMILY_SIGMA * np.random.default_rng(FAMILY_SEED + s).standard_normal(FAMILY_MODES)


def family_pencil(amplitudes: np.ndarray, nc: int = 500, b: int = 64) -> Pencil:
    """Member of the family with the given onsite amplitudes (chain recipe)."""
    return chain_pencil(nc, b, FAMILY_SEED, amplitudes=amplitudes, family_seed=FAMILY_SEED)


def onsite_modes(nc: int, modes: int = FAMILY_MODES) -> np.ndarray:
    """[nc][modes] values sin(k pi s_i) of the onsite field's Fourier modes."""
    s = (np.arange(nc) + 0.5) / nc
    return np.sin(np.pi * np.outer(s, np.arange(1, modes + 1)))


# Batched workload: independent uneven problems.  Problem p draws, from
# default_rng(BATCH_SEED + p): nc ~ U{50..200}, b from {32, 48, 64},
# M0 ~ U{16..64}; the pencil is the chain recipe with matrix seed
# BATCH_SEED + p, Ne = 16, and the interval holds round(0.6 M0) eigenvalues
# from index n // 4 (stored in tests/golden/intervals_batch.json).
BATCH_SEED = 3000
BATCH_NE = 16


def batch_shape(p: int) -> dict:
    rng = np.random.default_rng(BATCH_SEED + p)
    nc = int(rng.integers(50, 201))
    b = int(rng.choice([32, 48, 64]))
    m0 = int(rng.integers(16, 65))
    n = nc * b
    return dict(nc=nc, b=b, M0=m0, Ne=BATCH_NE, mseed=BATCH_SEED + p, yseed=BATCH_SEED + 500 + p,
                n_eig=int(round(0.6 * m0)), k0=n // 4)


# The batched configuration at its full shape: 256 problems, problem p draws
# from default_rng(BATCH_SEED + p) nc ~ U{50..500}, b from {32, 64, 96},
# M0 ~ U{16..64}; the chain recipe with matrix seed BATCH_SEED + p, Ne = 16,
# an interval of round(0.6 M0) eigenvalues from index n // 4
# (tests/golden/intervals_batch256.json).
BATCH256_COUNT = 256


def batch256_shape(p: int) -> dict:
    rng = np.random.default_rng([BATCH_SEED, 256, p])
    nc = int(rng.integers(50, 501))
    b = int(rng.choice([32, 64, 96]))
    m0 = int(rng.integers(16, 65))
    n = nc * b
    return dict(nc=nc, b=b, M0=m0, Ne=BATCH_NE, mseed=BATCH_SEED + p, yseed=BATCH_SEED + 500 + p,
                n_eig=int(round(0.6 * m0)), k0=n // 4)


def batch256_pencil(p: int) -> Pencil:
    s = batch256_shape(p)
    return chain_pencil(s["nc"], s["b"], s["mseed"])


def make_batch256(count: int, first: int = 0):
    """[(pencil, emin, emax, M0, Ne, Y0)] of batch256 problems first .. first+count-1."""
    with open(os.path.join(_GOLDEN, "intervals_batch256.json")) as f:
        iv = json.load(f)
    out = []
    for p in range(first, first + count):
        s = batch256_shape(p)
        e = iv[str(p)]
        pen = batch256_pencil(p)
        out.append((pen, float(e["emin"]), float(e["emax"]), s["M0"], s["Ne"],
                    random_subspace(pen.n, s["M0"], s["yseed"])))
    return out


def batch_pencil(p: int) -> Pencil:
    s = batch_shape(p)
    return chain_pencil(s["nc"], s["b"], s["mseed"])


def make_batch(count: int):
    """[(pencil, emin, emax, M0, Ne, Y0)] of the first ``count`` batch problems."""
    with open(os.path.join(_GOLDEN, "intervals_batch.json")) as f:
        iv = json.load(f)
    out = []
    for p in range(count):
        s = batch_shape(p)
        e = iv[str(p)]
        pen = batch_pencil(p)
        out.append((pen, float(e["emin"]), float(e["emax"]), s["M0"], s["Ne"],
                    random_subspace(pen.n, s["M0"], s["yseed"])))
    return out


def make_pencil(name: str) -> Pencil:
    w = WORKLOADS[name]
    if w["kind"] == "dense":
        return dense_random_pencil(w["nc"], w["b"], w["mseed"])
    if w["kind"] == "hchain":
        return hermitian_chain_pencil(w["nc"], w["b"], w["mseed"])
    if w["kind"] == "family":
        return chain_pencil(w["nc"], w["b"], w["mseed"], amplitudes=np.zeros(FAMILY_MODES),
                            family_seed=w["mseed"])
    return chain_pencil(w["nc"], w["b"], w["mseed"])


def load_interval(name: str) -> tuple[float, float]:
    """Search interval stored by tests/golden/make_intervals.py (oracle only)."""
    with open(os.path.join(_GOLDEN, "intervals.json")) as f:
        data = json.load(f)
    e = data[name]
    return float(e["emin"]), float(e["emax"])


def make_workload(name: str):
    """Return (pencil, emin, emax, M0, Ne, Y0) for a named workload."""
    w = WORKLOADS[name]
    p = make_pencil(name)
    emin, emax = load_interval(name)
    if w["kind"] == "hchain":
        Y0 = random_complex_subspace(p.n, w["M0"], w["yseed"])
    else:
        Y0 = random_subspace(p.n, w["M0"], w["yseed"])
    return p, emin, emax, w["M0"], w["Ne"], Y0
