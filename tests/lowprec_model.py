"""CPU model of reduced-precision arithmetic for the low-precision tests.

Test infrastructure (uses the oracle; never imported by the library).  It
rounds operands the way Sec. 5.2 and Alg. matmul describe: a value is
converted to the 16-bit format by round-to-nearest-even, error correction
splits a value x into x_hi = rnd(x) and x_lo = rnd((x - x_hi) 2^s) and
forms the product as hi*hi' + (lo*hi' + hi*lo') / 2^s, and "one can refine
one or both matrices" (Sec. 5.2): refining only the constant 1D matrix is
the matrix-side split.  Products accumulate exactly here (FP64), which
models the FP32 accumulator up to FP32 rounding.

Where the rounding sits follows the library's published contract (the
header: FP16/BF16 operands of every 1D contraction of the cell operator and
of the patch eigenvector transforms, FP32 elsewhere), so that the model's
failure modes can be compared with the GPU's.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

from oracle import multigrid, sipg

U32 = 2.0 ** -24
UNIT = {"f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}
SPLIT = {"f16": 2.0 ** 11, "bf16": 2.0 ** 8}


def round_f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def round_f16(a):
    """IEEE binary16, round to nearest even (numpy's conversion)."""
    return np.asarray(a, dtype=np.float64).astype(np.float16).astype(np.float64)


def round_bf16(a):
    """bfloat16 = the upper 16 bits of binary32, round to nearest even:
    add 0x7FFF plus the lowest kept bit, then clear the low 16 bits (the
    value is first rounded to binary32)."""
    b = np.asarray(a, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


ROUND = {"f32": round_f32, "f16": round_f16, "bf16": round_bf16}


def split(x, fmt):
    """Alg. matmul's hi / lo parts."""
    r = ROUND[fmt]
    hi = r(x)
    return hi, r((np.asarray(x) - hi) * SPLIT[fmt])


def effective_matrix(S, fmt, ec):
    """The matrix the products see: rnd(S) without correction, hi + lo/2^s
    when the matrix operand is refined (ec = 1 or 2)."""
    if fmt == "f32":
        return round_f32(S)
    hi, lo = split(S, fmt)
    return hi + lo / SPLIT[fmt] if ec in (1, 2) else hi


def matvec_lines(S, X, fmt, ec):
    """Y = S applied to every line (last axis) of X in the model arithmetic."""
    if fmt == "f32":
        return round_f32(X) @ round_f32(S).T
    Sh, Sl = split(S, fmt)
    Xh, Xl = split(X, fmt)
    Y = Xh @ Sh.T
    if ec in (1, 2):
        Y = Y + (Xh @ Sl.T) / SPLIT[fmt]
    if ec == 1:
        Y = Y + (Xl @ Sh.T) / SPLIT[fmt]
    return Y


def lowest_eigen_shift(n, k, fmt, ec):
    """Relative change of the smallest generalized eigenvalue of the 1D
    operator pair (L, M) of an n-cell line when their cell blocks are
    replaced by effective_matrix: how far the rounded operator moves the
    smoothest mode, which the V-cycle resolves through its coarse levels."""
    N = k + 1
    M, L = sipg.global_1d(n, k)
    M, L = M * n, L / n
    c = 1 if n >= 3 else 0
    Lc = L[c * N:(c + 1) * N, c * N:(c + 1) * N]
    Mc = M[:N, :N]
    eye = np.eye(n)
    Lr = L - np.kron(eye, Lc) + np.kron(eye, effective_matrix(Lc, fmt, ec))
    Mr = np.kron(eye, effective_matrix(Mc, fmt, ec))
    lam = sla.eigh(L, M, eigvals_only=True, subset_by_index=[0, 0])[0]
    lamr = sla.eigh(Lr, Mr, eigvals_only=True, subset_by_index=[0, 0])[0]
    return abs(lamr - lam) / lam


def data_unit(fmt, ec):
    """Relative rounding of the vector operand of a product."""
    if fmt == "f32":
        return 8 * U32
    return UNIT[fmt] ** 2 + 8 * U32 if ec == 1 else UNIT[fmt]


def _along(X, fn, axis):
    X = np.moveaxis(X, axis, -1)
    return np.moveaxis(fn(X), -1, axis)


class Level:
    """One mesh level in the model arithmetic: the cell-block part of the 1D
    operators through matvec_lines, the couplings between cells (face terms)
    and the boundary corrections exactly; the patch solve by fast
    diagonalization with every eigenvector transform through matvec_lines."""

    def __init__(self, n, k, fmt, ec):
        self.n, self.k, self.N, self.fmt, self.ec = n, k, k + 1, fmt, ec
        N = k + 1
        M, L = sipg.global_1d(n, k)
        M, L = M * n, L / n
        c = 1 if n >= 3 else 0
        Lc = L[c * N:(c + 1) * N, c * N:(c + 1) * N]
        self.Lc, self.Mc = Lc, M[:N, :N]
        self.Lrest = L - np.kron(np.eye(n), Lc)
        self.h = 1.0 / n
        self.fd = {}
        for v in range(1, n):
            key = (v == 1, v == n - 1)
            if key not in self.fd:
                sl = slice((v - 1) * N, (v + 1) * N)
                self.fd[key] = sla.eigh(L[sl, sl], M[sl, sl])

    def _blockwise(self, X, B):
        n, N = self.n, self.N
        shp = X.shape
        Y = matvec_lines(B, X.reshape(shp[:-1] + (n, N)), self.fmt, self.ec)
        return Y.reshape(shp)

    def _L(self, X, axis):
        return _along(X, lambda Y: self._blockwise(Y, self.Lc) + Y @ self.Lrest.T, axis)

    def _M(self, X, axis):
        return _along(X, lambda Y: self._blockwise(Y, self.Mc), axis)

    def apply(self, u):
        n, k = self.n, self.k
        U = sipg.to_tensor(u, n, k)
        t1, t2 = self._L(U, 2), self._M(U, 2)
        c = self._M(t1, 1) + self._L(t2, 1)
        e = self._M(t2, 1)
        return sipg.from_tensor(self.h * (self._M(c, 0) + self._L(e, 0)), n, k)

    def patch_correct(self, colour, r, x):
        n, k, N = self.n, self.k, self.N
        R = sipg.to_tensor(r, n, k)
        X = sipg.to_tensor(x, n, k).copy()
        mv = lambda S: (lambda Y: matvec_lines(S, Y, self.fmt, self.ec))
        for v, c in multigrid.vertex_patches(n):
            if c != colour:
                continue
            sl = [slice((v[d] - 1) * N, (v[d] + 1) * N) for d in range(3)]
            (lx, Sx), (ly, Sy), (lz, Sz) = [self.fd[(v[d] == 1, v[d] == n - 1)] for d in range(3)]
            P = R[sl[2], sl[1], sl[0]]
            P = _along(_along(_along(P, mv(Sx.T), 2), mv(Sy.T), 1), mv(Sz.T), 0)
            P = P / (self.h * (lz[:, None, None] + ly[None, :, None] + lx[None, None, :]))
            P = _along(_along(_along(P, mv(Sz), 0), mv(Sy), 1), mv(Sx), 2)
            X[sl[2], sl[1], sl[0]] += P
        return sipg.from_tensor(X, n, k)


class Hierarchy:
    """V(2,2) with the model levels, FP32 vectors, FP32 transfers and an
    exact coarse solve, entered with a power-of-two scaled right-hand side."""

    def __init__(self, n, k, fmt, ec):
        ns = [n]
        while ns[-1] > 2:
            ns.append(ns[-1] // 2)
        ns = ns[::-1]
        self.lev = [Level(m, k, fmt, ec) for m in ns]
        self.P = [None] + [multigrid.prolongation(ns[i - 1], k) for i in range(1, len(ns))]
        self.coarse = spla.splu(sipg.assemble(ns[0], k).tocsc())

    def smooth(self, l, x, b):
        L = self.lev[l]
        for _ in range(2):
            for c in range(8):
                x = round_f32(L.patch_correct(c, round_f32(b - L.apply(x)), x))
        return x

    def vcycle(self, l, x, b):
        if l == 0:
            return round_f32(self.coarse.solve(b))
        x = self.smooth(l, x, b)
        rc = round_f32(self.P[l].T @ round_f32(b - self.lev[l].apply(x)))
        x = round_f32(x + self.P[l] @ self.vcycle(l - 1, np.zeros(rc.shape), rc))
        return self.smooth(l, x, b)

    def precondition(self, v):
        s = 2.0 ** np.ceil(np.log2(np.abs(v).max()))
        return s * self.vcycle(len(self.lev) - 1, np.zeros(v.shape), round_f32(v / s))
