"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws random numbers and picks sizes; it holds none of the
method's arithmetic.  Inputs follow the paper's workloads: random vectors
(Sec. 5.2 uses N(0, 1); the apply benchmark uses U[-1, 1]) and manufactured
sine solutions on the unit cube (Sec. 7.2), plus sums of seeded sine modes
for the batched and learned workloads.
"""
import numpy as np


def uniform_vector(n_dofs, seed, low=-1.0, high=1.0):
    """FP64 vector with entries ~ U[low, high]."""
    return np.random.default_rng(seed).uniform(low, high, int(n_dofs))


def normal_vector(n_dofs, seed):
    """FP64 vector with entries ~ N(0, 1)."""
    return np.random.default_rng(seed).standard_normal(int(n_dofs))


def sine_modes(seed, n_modes=4, max_wavenumber=4):
    """Amplitudes a_m ~ U[-1, 1] and integer wavenumbers (p, q, r) ~
    U{1..max_wavenumber} of u = sum_m a_m sin(p pi x) sin(q pi y) sin(r pi z)."""
    rng = np.random.default_rng(seed)
    amps = rng.uniform(-1.0, 1.0, n_modes)
    pqr = rng.integers(1, max_wavenumber + 1, size=(n_modes, 3))
    return amps, pqr


def single_sine_modes():
    """The paper's u = sin(pi x) sin(pi y) sin(pi z)."""
    return np.array([1.0]), np.array([[1, 1, 1]])


def batch_problems(seed, count=64, edges=(16, 24, 32, 48, 64), degrees=(2, 3, 4, 5, 6, 7)):
    """(n, k) pairs of a batch of uneven problems."""
    rng = np.random.default_rng(seed)
    ns = rng.choice(np.asarray(edges), size=count)
    ks = rng.choice(np.asarray(degrees), size=count)
    return [(int(a), int(b)) for a, b in zip(ns, ks)]


def mesh_vertices(n, kind="identity", amplitude=0.0, seed=0, affine=None, shift=None):
    """Vertex positions of a structured mesh of n^3 hexahedra, array
    [n+1, n+1, n+1, 3] indexed [vz, vy, vx] (x, y, z last).

    kind "identity": the uniform grid of the unit cube.
    kind "smooth":   the grid moved by amplitude * s(x) * c, with
                     s = sin(pi x) sin(pi y) sin(pi z) (zero on the boundary)
                     and a seeded direction c in [-1, 1]^3.
    kind "jitter":   interior vertices moved by seeded offsets in
                     [-amplitude h, amplitude h]^3 (h = 1/n); boundary
                     vertices stay.
    Then x <- affine @ x + shift when given (a 3 x 3 matrix, a 3-vector)."""
    t = np.arange(n + 1, dtype=np.float64) / n
    Z, Y, X = np.meshgrid(t, t, t, indexing="ij")
    P = np.stack([X, Y, Z], axis=-1)
    rng = np.random.default_rng(seed)
    if kind == "smooth":
        c = rng.uniform(-1.0, 1.0, 3)
        s = np.sin(np.pi * X) * np.sin(np.pi * Y) * np.sin(np.pi * Z)
        P = P + amplitude * s[..., None] * c
    elif kind == "jitter":
        d = rng.uniform(-amplitude / n, amplitude / n, P.shape)
        inner = np.zeros(P.shape[:3], dtype=bool)
        inner[1:-1, 1:-1, 1:-1] = True
        P = P + d * inner[..., None]
    elif kind != "identity":
        raise ValueError("kind must be identity, smooth or jitter")
    if affine is not None:
        P = P @ np.asarray(affine, dtype=np.float64).T
    if shift is not None:
        P = P + np.asarray(shift, dtype=np.float64)
    return np.ascontiguousarray(P)


def rotation(seed):
    """A seeded proper rotation (QR of a Gaussian matrix, det +1)."""
    q, r = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q
