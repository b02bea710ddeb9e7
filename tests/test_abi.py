"""CPU checks of the boundary: the HIP library loads and exports every entry
point that include/sipg.h declares; the host-side 1D tables (compiled from
the library's own C++ source with g++, no GPU) agree with the oracle."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sipg.h")


def declared_entry_points():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sipg_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_entry_points()
    for must in ["sipg_create", "sipg_destroy", "sipg_apply", "sipg_smooth", "sipg_vcycle",
                 "sipg_fgmres", "sipg_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2407_09621_amd import sipg
    lib = sipg.load_library()
    missing = [n for n in declared_entry_points() if not hasattr(lib, n)]
    assert not missing, missing
    assert isinstance(lib.sipg_last_error(), bytes)


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2407_09621_amd import sipg
    with pytest.raises(FileNotFoundError):
        sipg.load_library(str(tmp_path / "missing.so"))


SHIM = r"""
#include "tables.h"
#include <cstring>
using namespace sipg;
extern "C" int shim_layout(int k, int n0, int* lay) {
  TableLayout L; build_device_table(k, n0, L);
  int v[] = {L.N, L.G, L.Gc, L.mass, L.lcell, L.d0, L.d1, L.gam, L.fd_s, L.fd_l,
             L.fdc_s, L.fdc_l, L.p1, L.total};
  std::memcpy(lay, v, sizeof(v)); return L.total; }
extern "C" void shim_table(int k, int n0, double* out) {
  TableLayout L; auto t = build_device_table(k, n0, L);
  std::memcpy(out, t.data(), t.size() * sizeof(double)); }
extern "C" int shim_even_odd(int k, double pen, double* out) {
  TableLayout L; auto t = build_device_table(k, 2, L, pen);
  if (L.N != 8) return -1;
  std::memcpy(out, t.data() + L.eo, 12 * 16 * sizeof(double)); return L.eo_ok; }
extern "C" void shim_extra(int k, int n0, int* out) {
  TableLayout L; build_device_table(k, n0, L);
  out[0] = L.eo; out[1] = L.eo_ok; out[2] = L.pw_l; out[3] = L.sym; out[4] = L.fd_eo;
  out[5] = L.fd_eo_ok; }
extern "C" void shim_offdiag(int k, double* lr, double* rl) {
  Tables1D t = make_tables_1d(k);
  std::memcpy(lr, t.lr.data(), t.lr.size() * 8); std::memcpy(rl, t.rl.data(), t.rl.size() * 8); }
"""


@pytest.fixture(scope="module")
def host_tables(tmp_path_factory):
    d = tmp_path_factory.mktemp("shim")
    src = d / "shim.cpp"
    src.write_text(SHIM)
    so = d / "shim.so"
    csrc = os.path.join(ROOT, "paper_2407_09621_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", csrc, str(src),
                    os.path.join(csrc, "tables.cpp"), "-o", str(so)], check=True)
    lib = ctypes.CDLL(str(so))

    def get(k, n0=2):
        lay = (ctypes.c_int * 14)()
        total = lib.shim_layout(k, n0, lay)
        keys = ["N", "G", "Gc", "mass", "lcell", "d0", "d1", "gam", "fd_s", "fd_l", "fdc_s",
                "fdc_l", "p1", "total"]
        L = dict(zip(keys, list(lay)))
        buf = np.zeros(total)
        lib.shim_table(k, n0, buf.ctypes.data_as(ctypes.c_void_p))
        N = k + 1
        lr = np.zeros(N * N)
        rl = np.zeros(N * N)
        lib.shim_offdiag(k, lr.ctypes.data_as(ctypes.c_void_p), rl.ctypes.data_as(ctypes.c_void_p))
        return L, buf, lr.reshape(N, N), rl.reshape(N, N)
    def extra(k, n0=2):
        out = (ctypes.c_int * 6)()
        lib.shim_extra(k, n0, out)
        return dict(zip(["eo", "eo_ok", "pw_l", "sym", "fd_eo", "fd_eo_ok"], list(out)))
    get.lib = lib
    get.layout_extra = extra
    return get


@pytest.mark.parametrize("k", range(1, 8))
def test_host_tables_match_oracle(host_tables, k):
    from oracle import basis1d, sipg as osipg
    L, t, lr, rl = host_tables(k, 3)
    N = k + 1
    Mh, Kh = basis1d.mass_stiffness(k)
    np.testing.assert_allclose(t[L["mass"]:L["mass"] + N * N].reshape(N, N), Mh, atol=1e-13)
    s0, s1, d0, d1 = basis1d.end_vectors(k)
    np.testing.assert_allclose(t[L["d0"]:L["d0"] + N], d0, atol=1e-10 * np.abs(d0).max())
    np.testing.assert_allclose(t[L["d1"]:L["d1"] + N], d1, atol=1e-10 * np.abs(d1).max())
    # cell blocks and couplings against the oracle's global 1D matrix (h = 1)
    for n in (1, 3):
        M, Lg = osipg.global_1d(n, k)
        Lg = Lg / n  # h-free
        blocks = t[L["lcell"]:L["lcell"] + 4 * N * N].reshape(4, N, N)
        if n == 1:
            np.testing.assert_allclose(blocks[3], Lg, atol=1e-10 * np.abs(Lg).max())
        else:
            sc = np.abs(Lg).max() * 1e-11
            np.testing.assert_allclose(blocks[1], Lg[:N, :N], atol=sc)
            np.testing.assert_allclose(blocks[0], Lg[N:2 * N, N:2 * N], atol=sc)
            np.testing.assert_allclose(blocks[2], Lg[2 * N:, 2 * N:], atol=sc)
            np.testing.assert_allclose(lr, Lg[:N, N:2 * N], atol=sc)
            np.testing.assert_allclose(rl, Lg[N:2 * N, :N], atol=sc)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_host_fast_diagonalization_pairs(host_tables, k):
    """S^T M_P S = I and S^T L_P S = diag(lam) for the four patch types and
    the coarse grid, with M_P, L_P from the oracle's global 1D matrices."""
    from oracle import sipg as osipg
    for n0 in (1, 2, 3):
        L, t, _, _ = host_tables(k, n0)
        N, G, Gc = L["N"], L["G"], L["Gc"]
        for typ in range(4):
            # a line of 4 cells; the patch is cells (1,2) with boundary flags
            n = 2 + (0 if typ & 1 else 1) + (0 if typ & 2 else 1)
            first = 0 if typ & 1 else 1
            M, Lg = osipg.global_1d(n, k)
            sl = slice(first * N, (first + 2) * N)
            Mp, Lp = M[sl, sl] * n, Lg[sl, sl] / n
            S = t[L["fd_s"] + typ * G * G:L["fd_s"] + (typ + 1) * G * G].reshape(G, G)
            lam = t[L["fd_l"] + typ * G:L["fd_l"] + (typ + 1) * G]
            np.testing.assert_allclose(S.T @ Mp @ S, np.eye(G), atol=1e-9)
            np.testing.assert_allclose(S.T @ Lp @ S, np.diag(lam), atol=1e-9 * np.abs(lam).max())
        M, Lg = osipg.global_1d(n0, k)
        S = t[L["fdc_s"]:L["fdc_s"] + Gc * Gc].reshape(Gc, Gc)
        lam = t[L["fdc_l"]:L["fdc_l"] + Gc]
        np.testing.assert_allclose(S.T @ (M * n0) @ S, np.eye(Gc), atol=1e-9)
        np.testing.assert_allclose(S.T @ (Lg / n0) @ S, np.diag(lam), atol=1e-9 * np.abs(lam).max())


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 7])
def test_host_even_odd_patch_diagonalization(host_tables, k):
    """The interior patch type in even-odd form: the eigenvectors rebuilt
    from YE, YO (s = [y; J y] / sqrt 2 and [y; -J y] / sqrt 2) diagonalise
    the oracle's interior patch pencil, S^T M_P S = I and
    S^T L_P S = diag(lamE, lamO), and the even-odd patch inverse
    S diag(1/lam) S^T equals L_P^{-1}."""
    from oracle import sipg as osipg
    L, t, _, _ = host_tables(k)
    X = host_tables.layout_extra(k)
    assert X["fd_eo_ok"] == 1
    N = k + 1
    G, H = 2 * N, N
    n = 4
    M, Lg = osipg.global_1d(n, k)
    sl = slice(N, 3 * N)  # cells 1 and 2 of 4: both faces interior
    Mp, Lp = M[sl, sl] * n, Lg[sl, sl] / n
    o = X["fd_eo"]
    YE = t[o:o + H * H].reshape(H, H)
    YO = t[o + H * H:o + 2 * H * H].reshape(H, H)
    lam = t[o + 2 * H * H:o + 2 * H * H + G]
    J = np.eye(H)[::-1]
    S = np.zeros((G, G))
    S[:H, :H], S[H:, :H] = YE, J @ YE
    S[:H, H:], S[H:, H:] = YO, -J @ YO
    np.testing.assert_allclose(S.T @ Mp @ S, np.eye(G), atol=1e-9)
    np.testing.assert_allclose(S.T @ Lp @ S, np.diag(lam), atol=1e-9 * np.abs(lam).max())
    Linv = np.linalg.inv(Lp)
    np.testing.assert_allclose(S @ np.diag(1.0 / lam) @ S.T, Linv,
                               atol=1e-9 * np.abs(Linv).max())


@pytest.mark.parametrize("k", [1, 3, 6])
def test_host_prolongation_table(host_tables, k):
    from oracle import multigrid
    L, t, _, _ = host_tables(k)
    N = k + 1
    P1 = t[L["p1"]:L["p1"] + 2 * N * N].reshape(2 * N, N)
    # the 3D embedding of child (0,0,0) is P1[:N] (x) P1[:N] (x) P1[:N]
    E = multigrid._child_embedding(k, (1, 0, 1))
    K = np.kron(P1[N:], np.kron(P1[:N], P1[N:]))
    np.testing.assert_allclose(E, K, atol=1e-12)


def test_batch_rejects_mixed_precision_before_allocating():
    """A batch shares one V-cycle precision; the check runs before any
    device call, so it holds without a GPU."""
    from paper_2407_09621_amd import SipgError
    from paper_2407_09621_amd import sipg as binding
    cfgs = (binding.Config * 2)()
    cfgs[0] = binding.Config(2, 4, 0, binding.PRECISION["f64"], 0, 2, 2)
    cfgs[1] = binding.Config(2, 4, 0, binding.PRECISION["f16"], 1, 2, 2)
    h = ctypes.c_void_p()
    with pytest.raises(SipgError, match="share precision"):
        binding._check(binding.load_library().sipg_batch_create(cfgs, 2, None, ctypes.byref(h)))
    assert not h.value


@pytest.mark.parametrize("kw,status,msg", [
    (dict(k=5, mg_precision="bf16", error_correction=0), 2, "stalls"),
    (dict(k=7, mg_precision="bf16", error_correction=0), 2, "stalls"),
    (dict(k=3, error_correction=3), 1, "error_correction"),
    (dict(k=3, penalty_scale=0.5), 1, "penalty_scale"),
    (dict(k=3, mg_precision="f16", smoother="additive"), 2, "additive"),
    (dict(k=0), 1, "k must be"),
])
def test_create_rejects_before_any_device_call(kw, status, msg):
    """Argument checks of sipg_create that run before any device call (so
    they hold without a GPU): the refused BF16 V-cycle without correction at
    k >= 5, EC modes, the penalty scale and the additive smoother's
    precision."""
    from paper_2407_09621_amd import sipg as binding
    args = dict(k=3, n_cells=4)
    args.update(kw)
    cfg = binding.make_config(**args)
    h = ctypes.c_void_p()
    st = binding.load_library().sipg_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert st == status and not h.value
    assert msg in binding.load_library().sipg_last_error().decode()


def test_create_rejects_half_an_allocator():
    from paper_2407_09621_amd import sipg as binding
    cfg = binding.make_config(3, 4)
    cfg.alloc = binding.TORCH_ALLOC
    h = ctypes.c_void_p()
    st = binding.load_library().sipg_create(ctypes.byref(cfg), None, ctypes.byref(h))
    assert st == 1 and not h.value
    assert "together" in binding.load_library().sipg_last_error().decode()


def test_header_and_binding_agree_on_struct_layouts():
    """The ctypes mirrors of the header's structs: field count and order of
    sipg_config, sipg_solve_opts and sipg_cnn_train_opts (sizes follow from
    the types)."""
    from paper_2407_09621_amd import sipg as binding
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    for cname, pyname in (("sipg_config", "Config"), ("sipg_solve_opts", "SolveOpts"),
                          ("sipg_cnn_train_opts", "CnnTrainOpts")):
        body = re.search(r"typedef struct \{([^{}]*)\} " + cname + ";", text).group(1)
        fields = re.findall(r"(\w+);", body)
        assert fields == [f[0] for f in getattr(binding, pyname)._fields_], cname


def _even_odd_model(blocks, u, n, h):
    """Degree-7 operator applied by the mirror-pair (even-odd) scheme of the
    matrix-core kernel, written with numpy on whole cells: E/O splits,
    one 4 x 4 block per half for the J-symmetric mass and cell blocks, the
    two couplings through S = v_m + J v_p and D = v_m - J v_p, the boundary
    corrections in the coupling form, three inverse splits and the h scale."""
    B = blocks.reshape(12, 4, 4)
    Me, Mo, Le, Lo, Crl, Cb = B[0], B[1], B[2], B[3], B[4:8], B[8:12]
    lo, hi = np.arange(4), 7 - np.arange(4)
    U = u.reshape(n, n, n, 8, 8, 8)  # cz, cy, cx, l (z), j (y), i (x)

    def eo(T, ax):
        a, b = np.take(T, lo, axis=ax), np.take(T, hi, axis=ax)
        return np.concatenate([a + b, a - b], axis=ax)

    def uneo(T, ax):
        e, o = np.take(T, range(4), axis=ax), np.take(T, range(4, 8), axis=ax)
        out = np.empty_like(T)
        idx = [slice(None)] * T.ndim
        idx[ax] = lo
        out[tuple(idx)] = (e + o) / 2
        idx[ax] = hi
        out[tuple(idx)] = (e - o) / 2
        return out

    def mul(Q, T, ax):
        return np.moveaxis(np.tensordot(Q, T, axes=([1], [ax])), 0, ax)

    def sym(Qe, Qo, T, ax):
        e, o = np.take(T, range(4), axis=ax), np.take(T, range(4, 8), axis=ax)
        return np.concatenate([mul(Qe, e, ax), mul(Qo, o, ax)], axis=ax)

    def cpl(C, Um, Up, ax):
        S, D = Um + np.flip(Up, ax), Um - np.flip(Up, ax)
        E = mul(C[0], np.take(S, lo, axis=ax), ax) + mul(C[1], np.take(S, hi, axis=ax), ax)
        O = mul(C[2], np.take(D, lo, axis=ax), ax) + mul(C[3], np.take(D, hi, axis=ax), ax)
        return np.concatenate([E, O], axis=ax)

    V = np.zeros_like(U)
    z = np.zeros((8, 8, 8))
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                c = (cz, cy, cx)
                u0 = U[c]

                def nb(d, s):
                    q = list(c)
                    q[d] += s
                    return U[tuple(q)] if 0 <= q[d] < n else z

                def dirterm(d, ax):
                    w = sym(Le, Lo, eo(u0, ax), ax) + cpl(Crl, nb(d, -1), nb(d, 1), ax)
                    if c[d] in (0, n - 1):
                        w = w + cpl(Cb, u0 * (c[d] == 0), u0 * (c[d] == n - 1), ax)
                    return w
                # axes of a cell block: 0 = z, 1 = y, 2 = x
                w = eo(dirterm(0, 0), 2)
                w = eo(sym(Me, Mo, w, 2), 1)
                t3 = sym(Me, Mo, w, 1)
                s1 = sym(Me, Mo, eo(dirterm(2, 2), 1), 1)
                s2 = sym(Me, Mo, eo(dirterm(1, 1), 2), 2)
                t3 = t3 + sym(Me, Mo, eo(s1 + s2, 0), 0)
                V[c] = h * uneo(uneo(uneo(t3, 0), 1), 2)
    return V.reshape(-1)


@pytest.mark.parametrize("n,pen", [(1, 1.0), (2, 1.0), (3, 1.0), (3, 2.5)])
def test_even_odd_blocks_reproduce_the_operator(host_tables, n, pen):
    """The degree-7 even-odd blocks of the device table (built by the
    library's own host code) with the scheme the matrix-core kernel follows
    reproduce the oracle's A u, interior and boundary cells (n = 1 puts
    both boundaries on one cell), also at a scaled penalty; lower degrees
    have no such blocks."""
    import ctypes as ct
    from oracle import sipg as osipg
    lib = host_tables.lib
    lib.shim_even_odd.argtypes = [ct.c_int, ct.c_double, ct.c_void_p]
    out = np.zeros(12 * 16)
    assert lib.shim_even_odd(7, ct.c_double(pen), out.ctypes.data_as(ct.c_void_p)) == 1
    assert lib.shim_even_odd(5, ct.c_double(pen), out.ctypes.data_as(ct.c_void_p)) == -1
    lib.shim_even_odd(7, ct.c_double(pen), out.ctypes.data_as(ct.c_void_p))
    u = np.random.default_rng(n).uniform(-1, 1, n ** 3 * 512)
    v = _even_odd_model(out, u, n, 1.0 / n)
    ref = osipg.kron_apply(u, n, 7, penalty_scale=pen)
    assert np.linalg.norm(v - ref) / np.linalg.norm(ref) < 1e-13


@pytest.mark.parametrize("k", [1, 3, 7])
def test_host_window_matrices_match_oracle(host_tables, k):
    """The patch-wise evaluation's window matrices of the device table (four
    window types) against the oracle's windows of lines of 2 and 4 cells
    (h-free: L_w scaled by h)."""
    from oracle import sipg as osipg
    L, t, _, _ = host_tables(k, 2)
    lay = host_tables.layout_extra(k, 2)
    G = 2 * (k + 1)
    W = t[lay["pw_l"]:lay["pw_l"] + 4 * G * G].reshape(4, G, G)
    for n, w, typ in [(2, 1, 3), (4, 1, 1), (4, 2, 0), (4, 3, 2)]:
        _, Lw = osipg.patch_1d(n, k, w)
        np.testing.assert_allclose(W[typ], Lw / n, atol=1e-11 * np.abs(Lw / n).max())


@pytest.mark.parametrize("k", range(1, 8))
def test_host_even_odd_half_blocks(host_tables, k):
    """The vector kernels apply the mass matrix and the interior cell block
    through their even-odd half-blocks; rebuilt as y_a = (QE e)_a + (QO o)_a,
    y_{N-1-a} = (QE e)_a - (QO o)_a (middle row of odd N: (QE e)_mid) they
    reproduce Q x for the oracle's matrices (odd and even N)."""
    from oracle import basis1d, sipg as osipg
    L, t, _, _ = host_tables(k, 2)
    off = host_tables.layout_extra(k, 2)["sym"]
    N, P, PE = k + 1, (k + 1) // 2, (k + 2) // 2
    Mh, _ = basis1d.mass_stiffness(k)
    _, Lg = osipg.global_1d(3, k)
    Lint = Lg[N:2 * N, N:2 * N] / 3
    rng = np.random.default_rng(k)
    base = off
    for Q in (Mh, Lint):
        QE = t[base:base + PE * PE].reshape(PE, PE)
        QO = t[base + PE * PE:base + PE * PE + P * P].reshape(P, P)
        base += PE * PE + P * P
        x = rng.uniform(-1, 1, N)
        e = np.array([x[b] + x[N - 1 - b] for b in range(PE)])
        o = np.array([x[b] - x[N - 1 - b] for b in range(P)])
        ye, yo = QE @ e, QO @ o
        y = np.zeros(N)
        for a in range(P):
            y[a], y[N - 1 - a] = ye[a] + yo[a], ye[a] - yo[a]
        if N % 2:
            y[P] = ye[P]
        np.testing.assert_allclose(y, Q @ x, atol=1e-12 * np.abs(Q).max() * np.abs(x).sum())
