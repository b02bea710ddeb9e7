"""The SIPG Laplacian on a uniform Cartesian mesh of the unit cube.

Sec. 2, eq. bilinear_form: find u_h in V_h with

    sum_K int_K grad u . grad v
  + sum_e int_e ( gamma_e [[u]] . [[v]] - {grad u} . [[v]] - [[u]] . {grad v} )
  = int f v,

with the interior-penalty parameter gamma_e = k(k+1)(1/h+ + 1/h-).

Readings (the printed form is garbled in places):
* The printed face term averages the normal-weighted traces.  Read literally
  the scheme is inconsistent.  We take the standard SIPG form of the work the
  paper cites for the method (Arnold et al.): the jump
  [[v]] = v+ n+ + v- n- (a vector) and the average {w} = (w+ + w-)/2.
* On boundary faces the paper sets {v} = v; the jump is [[v]] = v n and the
  penalty uses the one adjacent cell on both sides, gamma = 2k(k+1)/h.
* Dirichlet data g = 0 (all manufactured solutions used vanish on the
  boundary).

Degree-of-freedom layout (shared convention with the GPU library, stated, not
shared code): cells are numbered c = cx + n*cy + n*n*cz, and inside a cell the
N^3 local index is i + N*j + N*N*l with direction 0 (x) fastest, as in the
index arithmetic of the paper's Appendix A.  Global index = c*N^3 + local.

Two independent derivations are provided:
* ``assemble``   builds the sparse matrix by 3D quadrature on cells and 2D
                 quadrature on faces with full 3D gradients and vector
                 normals, directly from the bilinear form.
* ``kron_apply`` applies A = M (x) M (x) L + M (x) L (x) M + L (x) M (x) M on
                 the global tensor grid (Sec. 2.1, eq. tensorproduct_3d),
                 with 1D face terms derived by hand.
Their agreement is a pin (tests/test_oracle_sipg.py).
"""
import numpy as np
import scipy.sparse as sp

from . import basis1d


def penalty_hat(k, penalty_scale=1.0):
    """h-free interior penalty 2k(k+1): gamma_e = k(k+1)(1/h + 1/h) (Sec. 2).
    ``penalty_scale`` multiplies it (a user choice of the penalty; the scheme
    stays symmetric for any value and coercive for values >= 1)."""
    return 2.0 * k * (k + 1) * penalty_scale


# ---------------------------------------------------------------------------
# Local matrices by quadrature (plain definition)
# ---------------------------------------------------------------------------

def _tensor_basis_at(k, pts, h):
    """Values and physical gradients of all N^3 tensor basis functions at
    points given in reference coordinates pts[q] = (xi0, xi1, xi2) of a cell
    of size h.  Returns val [Q, N^3], grad [Q, N^3, 3]."""
    nodes = basis1d.gll_nodes(k)
    N = k + 1
    pts = np.asarray(pts, dtype=np.float64)
    Vx = basis1d.lagrange_values(nodes, pts[:, 0])
    Vy = basis1d.lagrange_values(nodes, pts[:, 1])
    Vz = basis1d.lagrange_values(nodes, pts[:, 2])
    Dx = basis1d.lagrange_derivs(nodes, pts[:, 0]) / h
    Dy = basis1d.lagrange_derivs(nodes, pts[:, 1]) / h
    Dz = basis1d.lagrange_derivs(nodes, pts[:, 2]) / h
    Q = len(pts)
    val = np.zeros((Q, N ** 3))
    grad = np.zeros((Q, N ** 3, 3))
    for l in range(N):
        for j in range(N):
            for i in range(N):
                I = i + N * j + N * N * l
                val[:, I] = Vx[:, i] * Vy[:, j] * Vz[:, l]
                grad[:, I, 0] = Dx[:, i] * Vy[:, j] * Vz[:, l]
                grad[:, I, 1] = Vx[:, i] * Dy[:, j] * Vz[:, l]
                grad[:, I, 2] = Vx[:, i] * Vy[:, j] * Dz[:, l]
    return val, grad


def cell_matrix(k, h):
    """int_K grad phi_I . grad phi_J over one cell of size h with the tensor
    N^3-point Gauss rule (exact for these polynomials)."""
    N = k + 1
    x, w = basis1d.gauss_rule(N)
    P = np.array([(a, b, c) for c in x for b in x for a in x])
    W = np.array([wa * wb * wc for wc in w for wb in w for wa in w]) * h ** 3
    _, g = _tensor_basis_at(k, P, h)
    return sum(g[:, :, d].T @ (W[:, None] * g[:, :, d]) for d in range(3))


def _face_points(k, d, side):
    """Tensor Gauss points on the face xi_d = side (0 or 1) of the reference
    cell, and weights (reference, unit area)."""
    N = k + 1
    x, w = basis1d.gauss_rule(N)
    t = [a for a in range(3) if a != d]
    pts, wts = [], []
    for b_i, b in enumerate(x):
        for a_i, a in enumerate(x):
            p = [0.0, 0.0, 0.0]
            p[t[0]] = a
            p[t[1]] = b
            p[d] = float(side)
            pts.append(p)
            wts.append(w[a_i] * w[b_i])
    return np.array(pts), np.array(wts)


def interior_face_blocks(k, d, h, penalty_scale=1.0):
    """The four blocks of the interior-face bilinear form on a face with
    normal e_d between the lower cell K- and the upper cell K+ (both of size
    h).  Returns dict with keys ('-','-'), ('-','+'), ('+','-'), ('+','+'):
    block[(t, s)][I, J] = a_e(phi_J on K_s, phi_I on K_t)."""
    gamma = penalty_scale * k * (k + 1) * (1.0 / h + 1.0 / h)
    pm, wq = _face_points(k, d, 1.0)   # K- sees the face at xi_d = 1
    pp, _ = _face_points(k, d, 0.0)    # K+ sees it at xi_d = 0
    wq = wq * h * h
    vm, gm = _tensor_basis_at(k, pm, h)
    vp, gp = _tensor_basis_at(k, pp, h)
    n_minus = np.zeros(3)
    n_minus[d] = 1.0
    n_plus = -n_minus
    side = {'-': (vm, gm, n_minus), '+': (vp, gp, n_plus)}
    blocks = {}
    for t in '-+':
        vt, gt, nt = side[t]
        for s in '-+':
            vs, gs, ns = side[s]
            # [[phi_J]] = phi_J n_s, [[phi_I]] = phi_I n_t (vectors);
            # {grad phi} = grad phi / 2 on the side the function lives on.
            jump_jump = float(ns @ nt) * vs[:, None, :] * vt[:, :, None]     # [q,I,J]
            avg_u_jump_v = 0.5 * (gs @ nt)[:, None, :] * vt[:, :, None]
            jump_u_avg_v = 0.5 * vs[:, None, :] * (gt @ ns)[:, :, None]
            integrand = gamma * jump_jump - avg_u_jump_v - jump_u_avg_v
            blocks[(t, s)] = np.tensordot(wq, integrand, axes=(0, 0))
    return blocks


def boundary_face_block(k, d, side, h, penalty_scale=1.0):
    """Boundary face xi_d = side of a cell: {v} = v, [[v]] = v n with the
    outward normal n, gamma = 2k(k+1)/h (reading: mirror cell, h- = h+)."""
    gamma = penalty_scale * k * (k + 1) * (1.0 / h + 1.0 / h)
    p, wq = _face_points(k, d, float(side))
    wq = wq * h * h
    v, g = _tensor_basis_at(k, p, h)
    n = np.zeros(3)
    n[d] = 1.0 if side == 1 else -1.0
    gn = g @ n                                 # [q, N^3]
    integrand = (gamma * v[:, :, None] * v[:, None, :]
                 - v[:, :, None] * gn[:, None, :]
                 - gn[:, :, None] * v[:, None, :])
    return np.tensordot(wq, integrand, axes=(0, 0))


# ---------------------------------------------------------------------------
# Global assembly
# ---------------------------------------------------------------------------

def n_dofs(n, k):
    return n ** 3 * (k + 1) ** 3


def _coo_block(rows_base, cols_base, block):
    nb = block.shape[0]
    r = (rows_base[:, None, None] + np.arange(nb)[None, :, None])
    c = (cols_base[:, None, None] + np.arange(nb)[None, None, :])
    d = np.broadcast_to(block[None, :, :], r.shape[:1] + block.shape)
    r, c = np.broadcast_arrays(r, c)
    return r.ravel(), c.ravel(), d.ravel()


def assemble(n, k, boundary_terms=True, penalty_scale=1.0):
    """Sparse CSR matrix of the SIPG form on n^3 cells of size h = 1/n:
    cell loop, interior-face loop and boundary-face loop of the matrix-free
    skeleton in Sec. 2.1 (items (ii)(a)-(d)), with each local integral
    evaluated by quadrature.  ``boundary_terms=False`` drops the boundary-face
    integrals (used by the constant-annihilation pin)."""
    h = 1.0 / n
    N = k + 1
    nb = N ** 3
    cells = np.arange(n ** 3)
    cx, cy, cz = cells % n, (cells // n) % n, cells // (n * n)
    coord = [cx, cy, cz]
    stride = [1, n, n * n]
    R, C, D = [], [], []

    def add(rc, cc, blk):
        r, c, d = _coo_block(rc * nb, cc * nb, blk)
        R.append(r)
        C.append(c)
        D.append(d)

    add(cells, cells, cell_matrix(k, h))
    for d in range(3):
        blocks = interior_face_blocks(k, d, h, penalty_scale)
        lower = cells[coord[d] < n - 1]
        upper = lower + stride[d]
        add(lower, lower, blocks[('-', '-')])
        add(lower, upper, blocks[('-', '+')])
        add(upper, lower, blocks[('+', '-')])
        add(upper, upper, blocks[('+', '+')])
        if boundary_terms:
            add(cells[coord[d] == 0], cells[coord[d] == 0],
                boundary_face_block(k, d, 0, h, penalty_scale))
            add(cells[coord[d] == n - 1], cells[coord[d] == n - 1],
                boundary_face_block(k, d, 1, h, penalty_scale))
    R = np.concatenate(R)
    C = np.concatenate(C)
    D = np.concatenate(D)
    A = sp.coo_matrix((D, (R, C)), shape=(n_dofs(n, k),) * 2).tocsr()
    A.sum_duplicates()
    return A


# ---------------------------------------------------------------------------
# Second derivation: Kronecker sum on the global tensor grid
# ---------------------------------------------------------------------------

def global_1d(n, k, penalty_scale=1.0):
    """Global 1D matrices on the line of n cells, size nN x nN:
    M = h * blockdiag(Mhat) and L = (1/h) * (Khat blocks + 1D face terms).

    1D face terms of the form on a point face x_f between cell c (left) and
    c+1 (right), with traces u- = s1.u_c, u+ = s0.u_{c+1}, derivatives
    (1/h) d1.u_c and (1/h) d0.u_{c+1}, jump u- - u+ and average of the
    derivatives; boundary points use the outward normal (-1 at x = 0,
    +1 at x = 1)."""
    h = 1.0 / n
    N = k + 1
    Mh, Kh = basis1d.mass_stiffness(k)
    s0, s1, d0, d1 = basis1d.end_vectors(k)
    g = penalty_hat(k, penalty_scale)
    o = np.outer
    LL = g * o(s1, s1) - 0.5 * (o(s1, d1) + o(d1, s1))
    LR = -g * o(s1, s0) - 0.5 * o(s1, d0) + 0.5 * o(d1, s0)
    RL = -g * o(s0, s1) + 0.5 * o(s0, d1) - 0.5 * o(d0, s1)
    RR = g * o(s0, s0) + 0.5 * (o(s0, d0) + o(d0, s0))
    B0 = g * o(s0, s0) + (o(s0, d0) + o(d0, s0))
    B1 = g * o(s1, s1) - (o(s1, d1) + o(d1, s1))
    L = np.zeros((n * N, n * N))
    for c in range(n):
        L[c * N:(c + 1) * N, c * N:(c + 1) * N] += Kh
    for c in range(n - 1):
        a, b = slice(c * N, (c + 1) * N), slice((c + 1) * N, (c + 2) * N)
        L[a, a] += LL
        L[a, b] += LR
        L[b, a] += RL
        L[b, b] += RR
    L[0:N, 0:N] += B0
    L[(n - 1) * N:, (n - 1) * N:] += B1
    M = np.kron(np.eye(n), Mh)
    return h * M, L / h


def to_tensor(u, n, k):
    """Cell-blocked vector -> global tensor array U[Z, Y, X] with
    X = cx*N + i, Y = cy*N + j, Z = cz*N + l."""
    N = k + 1
    return (np.asarray(u).reshape(n, n, n, N, N, N)   # cz cy cx l j i
            .transpose(0, 3, 1, 4, 2, 5).reshape(n * N, n * N, n * N))


def from_tensor(U, n, k):
    N = k + 1
    return (np.asarray(U).reshape(n, N, n, N, n, N)    # cz l cy j cx i
            .transpose(0, 2, 4, 1, 3, 5).reshape(-1))


def _along(U, A, axis):
    """Apply the matrix A along one axis of the 3D array U."""
    U = np.moveaxis(U, axis, -1)
    shp = U.shape
    V = (A @ U.reshape(-1, shp[-1]).T).T
    return np.moveaxis(V.reshape(shp), -1, axis)


def kron_apply(u, n, k, penalty_scale=1.0):
    """v = A u with A = Mz(x)My(x)Lx + Mz(x)Ly(x)Mx + Lz(x)My(x)Mx applied
    factor by factor on the global tensor grid (eq. tensorproduct_3d)."""
    M, L = global_1d(n, k, penalty_scale)
    M = sp.csr_matrix(M)
    L = sp.csr_matrix(L)
    U = to_tensor(u, n, k)
    Mx = _along(U, M, 2)
    V = _along(_along(_along(U, L, 2), M, 1), M, 0)
    V += _along(_along(Mx, L, 1), M, 0)
    V += _along(_along(Mx, M, 1), L, 0)
    return from_tensor(V, n, k)


def patch_1d(n, k, w, penalty_scale=1.0):
    """Mass and stiffness-plus-face matrices (2N x 2N) of the 1D window w
    (cells w-1 and w, 1 <= w <= n-1) of a line of n cells, for the patch-wise
    evaluation of Sec. 2.1 (Fig. patch_int): the window carries the whole
    face integral of its interior face and, at the ends of the line, of the
    boundary face of its end cell; each cell integral (mass and stiffness)
    is shared by the windows that contain the cell (weight 1/2, or 1 for the
    first and last cell, which lie in one window only).  Summed over all
    windows they give the global M and L of global_1d."""
    if not (n >= 2 and 1 <= w <= n - 1):
        raise ValueError("windows exist for 1 <= w <= n - 1, n >= 2")
    h = 1.0 / n
    N = k + 1
    Mh, Kh = basis1d.mass_stiffness(k)
    s0, s1, d0, d1 = basis1d.end_vectors(k)
    g = penalty_hat(k, penalty_scale)
    o = np.outer
    a, b = w - 1, w
    wa = 1.0 if a == 0 else 0.5
    wb = 1.0 if b == n - 1 else 0.5
    L = np.zeros((2 * N, 2 * N))
    L[:N, :N] = wa * Kh + g * o(s1, s1) - 0.5 * (o(s1, d1) + o(d1, s1))
    L[:N, N:] = -g * o(s1, s0) - 0.5 * o(s1, d0) + 0.5 * o(d1, s0)
    L[N:, :N] = -g * o(s0, s1) + 0.5 * o(s0, d1) - 0.5 * o(d0, s1)
    L[N:, N:] = wb * Kh + g * o(s0, s0) + 0.5 * (o(s0, d0) + o(d0, s0))
    if a == 0:
        L[:N, :N] += g * o(s0, s0) + (o(s0, d0) + o(d0, s0))
    if b == n - 1:
        L[N:, N:] += g * o(s1, s1) - (o(s1, d1) + o(d1, s1))
    M = np.zeros((2 * N, 2 * N))
    M[:N, :N] = wa * Mh
    M[N:, N:] = wb * Mh
    return h * M, L / h


def patchwise_apply(u, n, k, penalty_scale=1.0):
    """v = A u evaluated patch by patch (Sec. 2.1, Fig. patch_int): for every
    interior vertex (wx, wy, wz) the 2x2x2-cell patch applies its own
    Kronecker sum Mz (x) My (x) Lx + Mz (x) Ly (x) Mx + Lz (x) My (x) Mx of
    the window matrices (patch_1d) to the patch's (2N)^3 coefficients, and
    the results are summed into v.  Because every window matrix sum gives
    the global 1D matrices, the sum over patches is A u exactly."""
    N = k + 1
    U = to_tensor(u, n, k)
    V = np.zeros_like(U)
    mats = [patch_1d(n, k, w, penalty_scale) for w in range(1, n)]
    for wz in range(1, n):
        Mz, Lz = mats[wz - 1]
        for wy in range(1, n):
            My, Ly = mats[wy - 1]
            for wx in range(1, n):
                Mx, Lx = mats[wx - 1]
                sl = (slice((wz - 1) * N, (wz + 1) * N), slice((wy - 1) * N, (wy + 1) * N),
                      slice((wx - 1) * N, (wx + 1) * N))
                P = U[sl]
                Q = _along(_along(_along(P, Lx, 2), My, 1), Mz, 0)
                Q += _along(_along(_along(P, Mx, 2), Ly, 1), Mz, 0)
                Q += _along(_along(_along(P, Mx, 2), My, 1), Lz, 0)
                V[sl] += Q
    return from_tensor(V, n, k)


def apply_rows(u, n, k, rows):
    """(A u)_r for selected global rows r, from the local quadrature
    matrices: cell block plus the face blocks of the row's cell.  Used to
    sample large outputs one by one."""
    h = 1.0 / n
    N = k + 1
    nb = N ** 3
    u = np.asarray(u)
    Ac = cell_matrix(k, h)
    faces = [interior_face_blocks(k, d, h) for d in range(3)]
    bnd = [[boundary_face_block(k, d, s, h) for s in (0, 1)] for d in range(3)]
    stride = [1, n, n * n]
    out = np.zeros(len(rows))
    for t, r in enumerate(rows):
        c, I = divmod(int(r), nb)
        co = [c % n, (c // n) % n, c // (n * n)]
        acc = Ac[I] @ u[c * nb:(c + 1) * nb]
        for d in range(3):
            if co[d] > 0:   # this cell is the upper cell of the lower face
                cm = c - stride[d]
                acc += faces[d][('+', '+')][I] @ u[c * nb:(c + 1) * nb]
                acc += faces[d][('+', '-')][I] @ u[cm * nb:(cm + 1) * nb]
            else:
                acc += bnd[d][0][I] @ u[c * nb:(c + 1) * nb]
            if co[d] < n - 1:
                cp = c + stride[d]
                acc += faces[d][('-', '-')][I] @ u[c * nb:(c + 1) * nb]
                acc += faces[d][('-', '+')][I] @ u[cp * nb:(cp + 1) * nb]
            else:
                acc += bnd[d][1][I] @ u[c * nb:(c + 1) * nb]
        out[t] = acc
    return out


def node_coordinates(n, k):
    """Physical coordinates [n_dofs, 3] of every DoF (its GLL node)."""
    N = k + 1
    h = 1.0 / n
    x = basis1d.gll_nodes(k)
    cells = np.arange(n ** 3)
    cx, cy, cz = cells % n, (cells // n) % n, cells // (n * n)
    loc = np.arange(N ** 3)
    i, j, l = loc % N, (loc // N) % N, loc // (N * N)
    X = (cx[:, None] + x[i][None, :]) * h
    Y = (cy[:, None] + x[j][None, :]) * h
    Z = (cz[:, None] + x[l][None, :]) * h
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
