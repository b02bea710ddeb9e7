"""Pins of the oracle's learned-stage functions against facts fixed outside
the oracle: node coordinates, scipy's n-d correlation, closed forms of
shifts and of Adam under a constant gradient, central finite differences,
and the exact-correction limit of the preconditioner."""
import numpy as np
import pytest
import scipy.ndimage as ndi
import scipy.sparse.linalg as spla

from oracle import learned as L
from oracle import multigrid, rhs, sipg
from paper_2407_09621_amd import inputs


@pytest.mark.parametrize("k,n", [(1, 2), (3, 2), (2, 3)])
def test_grid_mapping_follows_node_coordinates(k, n):
    """Grid axes run along the physical axes: gx orders the x coordinate of
    the nodes, and a grid point's coordinates do not depend on the other two
    grid indices."""
    X = sipg.node_coordinates(n, k)
    G = n * (k + 1)
    gx, gy, gz = (L.cells_to_grid(X[:, d], n, k) for d in range(3))
    for c, axis in ((gx, 2), (gy, 1), (gz, 0)):
        assert np.all(np.diff(c, axis=axis) >= -1e-15)          # monotone along its axis
        for other in {0, 1, 2} - {axis}:
            assert np.allclose(np.diff(c, axis=other), 0.0)     # constant across others
    assert gx.shape == (G, G, G)
    u = np.arange(X.shape[0], dtype=float)
    assert np.array_equal(L.grid_to_cells(L.cells_to_grid(u, n, k), n, k), u)


def test_grid_mapping_explicit_loop():
    n, k = 2, 2
    N, G = k + 1, 2 * (k + 1)
    u = np.arange(n ** 3 * N ** 3, dtype=float)
    g = L.cells_to_grid(u, n, k)
    for cz in range(n):
        for cy in range(n):
            for cx in range(n):
                for l in range(N):
                    for j in range(N):
                        for i in range(N):
                            idx = (cx + n * cy + n * n * cz) * N ** 3 + i + N * j + N * N * l
                            assert g[N * cz + l, N * cy + j, N * cx + i] == u[idx]
    assert g.shape == (G, G, G)


def test_conv3d_equals_scipy_correlate():
    rng = np.random.default_rng(1)
    cin, cout, G = 3, 2, 6
    x = rng.standard_normal((cin, G, G, G))
    w = rng.standard_normal((cout, cin, 3, 3, 3))
    b = rng.standard_normal(cout)
    y = L.conv3d(x, w, b)
    for co in range(cout):
        ref = b[co] + sum(ndi.correlate(x[ci], w[co, ci], mode="constant", cval=0.0)
                          for ci in range(cin))
        assert np.allclose(y[co], ref, rtol=1e-13, atol=1e-13)


def test_conv3d_delta_kernel_is_a_zero_filled_shift():
    rng = np.random.default_rng(2)
    G = 5
    x = rng.standard_normal((1, G, G, G))
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 2, 0, 1] = 1.0            # offset (dz, dy, dx) = (+1, -1, 0)
    y = L.conv3d(x, w, np.zeros(1))[0]
    ref = np.zeros((G, G, G))
    ref[:G - 1, 1:, :] = x[0, 1:, :G - 1, :]
    assert np.array_equal(y, ref)


def _tiny_net(C, seed):
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in L.param_shapes(C).items():
        p[name] = rng.standard_normal(shp) * (0.4 if name.startswith("w") else 0.2)
    return p


def test_gradients_match_central_differences():
    """Every parameter's exact gradient against central differences of the
    masked loss (FP64, h = 1e-6), on a batch of two 4^3 grids, 3 channels."""
    C, G, sigma = 3, 4, 0.5
    rng = np.random.default_rng(3)
    params = _tiny_net(C, 4)
    xs = [rng.standard_normal((G, G, G)) for _ in range(2)]
    ts = [rng.standard_normal((G, G, G)) for _ in range(2)]
    ms = [rng.uniform(0, 1, (G, G, G)) for _ in range(2)]
    loss, grads = L.loss_and_grads(params, sigma, xs, ts, ms)
    flat = L.flatten(params)
    gflat = L.flatten(grads)

    def f(th):
        return L.loss_and_grads(L.unflatten(th, C), sigma, xs, ts, ms)[0]

    assert abs(f(flat) - loss) < 1e-14 * max(1.0, loss)
    idx = rng.choice(flat.size, 60, replace=False)
    idx = np.concatenate([idx, [flat.size - 1, 0]])
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = 1e-6
        fd = (f(flat + e) - f(flat - e)) / 2e-6
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(gflat[i])), (i, fd, gflat[i])


def test_mse_closed_form_and_zero_mask_points():
    rng = np.random.default_rng(5)
    G = 4
    y, t = rng.standard_normal((G, G, G)), rng.standard_normal((G, G, G))
    m = np.zeros((G, G, G))
    m[1:3, 1:3, 1:3] = 1.0
    assert np.isclose(L.masked_mse(y, t, m, 2.0), np.mean((2 * y[1:3, 1:3, 1:3] - t[1:3, 1:3, 1:3]) ** 2))


def test_adam_constant_gradient_closed_form():
    """With a constant gradient the bias-corrected moments equal g and g^2,
    so every step moves by lr g / (|g| + eps)."""
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    opt = L.Adam(4, lr=0.01)
    th = np.zeros(4)
    for _ in range(7):
        th = opt.step(th, g)
    assert np.allclose(th, -7 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)


def test_adam_first_step_then_sign_flip():
    opt = L.Adam(1, lr=0.1, beta1=0.5, beta2=0.75, eps=0.0)
    th = opt.step(np.zeros(1), np.array([2.0]))
    assert np.isclose(th[0], -0.1)
    # step 2: m = .5*2*.5 + .5*(-2) ... written out: m = 0.5 m1 + 0.5 g2
    th2 = opt.step(th, np.array([-2.0]))
    m = 0.5 * (0.5 * 2.0) + 0.5 * (-2.0)
    v = 0.75 * (0.25 * 4.0) + 0.25 * 4.0
    assert np.isclose(th2[0], th[0] - 0.1 * (m / 0.75) / np.sqrt(v / (1 - 0.75 ** 2)))


def test_crop_mask_radius():
    G, c = 12, 8
    # along z: low face is the grid's face (kept), high face interior (4 dropped)
    assert list(L.crop_mask(G, (0, 0, 0), c)[:, 0, 0]) == [1, 1, 1, 1, 0, 0, 0, 0]
    # along y: both faces interior, nothing survives
    assert not L.crop_mask(G, (0, 2, 0), c).any()
    # along x: low face interior, high face the grid's face
    assert list(L.crop_mask(G, (0, 0, 4), c)[0, 0, :]) == [0, 0, 0, 0, 1, 1, 1, 1]
    assert L.crop_mask(G, (0, 0, 0), G).all()


def test_crop_mask_keeps_exactly_the_unchanged_outputs():
    """Where the mask is 1 the network output on the crop equals the output
    on the full grid (receptive radius 4 for four 3^3 layers)."""
    C, G, c = 2, 14, 10
    p = _tiny_net(C, 6)
    x = np.random.default_rng(7).standard_normal((G, G, G))
    full = L.forward(p, x)[0]
    for off in [(0, 4, 2), (4, 0, 4), (2, 2, 2)]:
        part = L.forward(p, L.crop(x, off, c))[0]
        m = L.crop_mask(G, off, c)
        ref = L.crop(full, off, c)
        assert np.allclose(part[m > 0], ref[m > 0], rtol=1e-12, atol=1e-12)
        # and the radius is tight: one point closer differs somewhere
        m3 = L.crop_mask(G, off, c, radius=3)
        assert not np.allclose(part[m3 > 0], ref[m3 > 0], rtol=1e-12, atol=1e-12)


def test_pow2_ceil():
    for v, r in [(1.0, 1.0), (0.75, 1.0), (0.5, 0.5), (3.0, 4.0), (1e-300, 2.0 ** -996)]:
        assert L.pow2_ceil(v) == r
    for v in np.random.default_rng(8).uniform(1e-6, 1e6, 100):
        s = L.pow2_ceil(v)
        assert s / 2 < v <= s


def test_pairs_satisfy_the_error_equation():
    """rho = A e for every pair (to rounding); rho / s lies in [-1, 1] with
    max |.| > 1/2."""
    n, k = 4, 2
    H = multigrid.Hierarchy(n, k)
    A = H.levels[-1].A
    amps, pqr = inputs.sine_modes(11)
    b = rhs.rhs(rhs.SineModes(amps, pqr), n, k)
    x = spla.spsolve(A.tocsc(), b)
    pairs = L.make_pairs(A, H.precondition, x, 3, n, k)
    absA = abs(A)
    for rg, eg, s in pairs:
        rho, e = L.grid_to_cells(rg, n, k), L.grid_to_cells(eg, n, k)
        # rho = A x - A z and e = x - z cancel; rounding is eps-relative to |A||x|
        assert np.linalg.norm(A @ e - rho) < 1e-13 * np.linalg.norm(absA @ np.abs(x)) / s
        assert 0.5 < np.abs(rho).max() <= 1.0
        x = e * s / L.pow2_ceil(np.abs(e * s).max())
    # the chain's next start is the previous error: e_1 / s_1 is the V-cycle
    # error of x_1 = e_0 / 2^ceil(log2 max|e_0|)
    e0 = L.grid_to_cells(pairs[0][1], n, k) * pairs[0][2]
    x1 = e0 / L.pow2_ceil(np.abs(e0).max())
    r1 = A @ x1
    e1 = x1 - H.precondition(r1)
    assert np.allclose(L.grid_to_cells(pairs[1][1], n, k) * pairs[1][2], e1, rtol=1e-12, atol=1e-14)


def test_exact_correction_converges_in_one_iteration():
    """With a 'network' that returns the exact scaled error, the stage
    yields A^{-1} v, so FGMRES converges in one iteration; with a zero
    network the solve is the plain multigrid solve."""
    n, k = 4, 2
    H = multigrid.Hierarchy(n, k)
    A = H.levels[-1].A
    lu = spla.splu(A.tocsc())
    amps, pqr = inputs.sine_modes(12)
    b = rhs.rhs(rhs.SineModes(amps, pqr), n, k)
    seen = {}

    def exact(grid_rho):
        rho = L.grid_to_cells(grid_rho, n, k)
        seen["n"] = seen.get("n", 0) + 1
        return L.cells_to_grid(lu.solve(rho), n, k)

    x, info = L.solve(A, b, H.precondition, exact, n, k, rtol=1e-10)
    assert info["iterations"] == 1 and not info["fell_back"] and seen["n"] == 1
    x0, i0 = L.solve(A, b, H.precondition, lambda g: np.zeros_like(g), n, k, rtol=1e-10)
    from oracle import fgmres as ofg
    xp, ip = ofg.fgmres(lambda v: A @ v, b, H.precondition, rtol=1e-10)
    assert i0["iterations"] == ip["iterations"] and np.allclose(x0, xp, rtol=1e-12, atol=1e-14)


def test_fallback_on_stagnation_and_non_finite():
    n, k = 4, 2
    H = multigrid.Hierarchy(n, k)
    A = H.levels[-1].A
    amps, pqr = inputs.sine_modes(13)
    b = rhs.rhs(rhs.SineModes(amps, pqr), n, k)
    rng = np.random.default_rng(14)
    noisy = lambda g: 1e9 * rng.standard_normal(g.shape)
    # the residual-minimising factor keeps even a useless correction harmless
    x, info = L.solve(A, b, H.precondition, noisy, n, k, rtol=1e-10)
    assert not info["fell_back"] and info["rel_res_true"] < 1e-9
    xp, ip = L.solve(A, b, H.precondition, lambda g: np.zeros_like(g), n, k, rtol=1e-10)
    assert info["iterations"] <= ip["iterations"] + 1
    # a threshold no iteration can meet forces the stagnation switch
    x, info = L.solve(A, b, H.precondition, noisy, n, k, rtol=1e-10, stagnation=1e-12)
    assert info["fell_back"] and info["rel_res_true"] < 1e-9
    bad = lambda g: np.full(g.shape, np.nan)
    x, info = L.solve(A, b, H.precondition, bad, n, k, rtol=1e-10)
    assert info["fell_back"] and info["rel_res_true"] < 1e-9


def test_residual_loss_gradients_match_central_differences():
    """The residual-aware loss min_alpha ||rho - alpha A c||^2 / ||rho||^2
    (c = sigma net(rho) in cells, A the SIPG operator of a 2^3 mesh of
    degree 1, 4^3 grid): every sampled parameter's exact gradient against
    central differences, and the loss against a brute-force minimisation
    over alpha."""
    C, n, k, sigma = 3, 2, 1, 0.25
    rng = np.random.default_rng(5)
    params = _tiny_net(C, 6)
    A = sipg.assemble(n, k)
    G = n * (k + 1)
    rhos = [rng.standard_normal((G, G, G)) for _ in range(2)]
    loss, grads = L.residual_loss_and_grads(params, sigma, A, rhos, n, k)
    from scipy.optimize import minimize_scalar
    num = 0.0
    for g in rhos:
        c = sigma * L.grid_to_cells(L.forward(params, g)[0], n, k)
        rho = L.grid_to_cells(g, n, k)
        q = A @ c
        best = minimize_scalar(lambda a: float(np.sum((rho - a * q) ** 2)),
                               bracket=(-10.0, 10.0), tol=1e-12)
        num += best.fun
    den = sum(float(np.sum(g * g)) for g in rhos)
    assert abs(loss - num / den) < 1e-10 * max(1.0, loss)
    # no dependence on the output scale: alpha absorbs it
    assert abs(L.residual_loss_and_grads(params, 4.0 * sigma, A, rhos, n, k)[0] - loss) \
        < 1e-13 * max(1.0, loss)
    flat, gflat = L.flatten(params), L.flatten(grads)

    def f(th):
        return L.residual_loss_and_grads(L.unflatten(th, C), sigma, A, rhos, n, k)[0]

    idx = np.concatenate([rng.choice(flat.size, 60, replace=False), [flat.size - 1, 0]])
    for i in idx:
        e = np.zeros_like(flat)
        e[i] = 1e-6
        fd = (f(flat + e) - f(flat - e)) / 2e-6
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(gflat[i])), (i, fd, gflat[i])


def test_residual_loss_is_zero_for_the_exact_correction():
    """A network whose output is the exact error A^{-1} rho (a linear map, here
    emulated by a zero network plus the closed form) leaves no residual: the
    loss of c = A^{-1} rho is 0 (the step length is 1) and of c = 0 is 1
    (q = 0: step length 0)."""
    n, k = 2, 1
    A = sipg.assemble(n, k).toarray()
    rho = np.random.default_rng(1).standard_normal(A.shape[0])
    c = np.linalg.solve(A, rho)
    assert np.linalg.norm(rho - A @ c) ** 2 / (rho @ rho) < 1e-24
    params = {key: np.zeros(shp) for key, shp in L.param_shapes(2).items()}
    loss, _ = L.residual_loss_and_grads(params, 1.0, A, [L.cells_to_grid(rho, n, k)], n, k)
    assert abs(loss - 1.0) < 1e-15
