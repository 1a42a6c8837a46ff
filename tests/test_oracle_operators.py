"""Pins of the forward operators of ``oracle.operators`` (CPU): exactness on polynomials at every
level of a refined layout, cells at the refinement interface included (there the neighbour is the
parent's quadratic, exact for quadratics), curl of a gradient = 0, and consistency with the
refined solve."""
import numpy as np

from oracle import multires, operators
from test_oracle_multires import gaussian_problem

N_B = 8


def refined_layout():
    """2 x 2 x 2 base blocks, base block (1, 0, 1) refined into its 8 children."""
    base = [(i, j, k) for k in range(2) for j in range(2) for i in range(2)]
    fine = [(2 + a, 0 + b, 2 + c) for c in range(2) for b in range(2) for a in range(2)]
    blocks = np.array(base + fine, dtype=np.int32)
    levels = np.array([0] * 8 + [1] * 8, dtype=np.int32)
    return blocks, levels


def positions(blocks, levels, n_b):
    """Cell-centre coordinates (x, y, z) in base cells, each [n, z, y, x]."""
    n = len(blocks)
    g = np.arange(n_b) + 0.5
    P = np.zeros((3, n, n_b, n_b, n_b))
    for i in range(n):
        h = 2.0 ** (-int(levels[i]))
        z, y, x = np.meshgrid((blocks[i][2] * n_b + g) * h, (blocks[i][1] * n_b + g) * h,
                              (blocks[i][0] * n_b + g) * h, indexing="ij")
        P[0, i], P[1, i], P[2, i] = x, y, z
    return P


def _check_on_mask(got, exact, mask, rel=1e-12):
    scale = max(np.abs(exact[..., mask] if exact.ndim > mask.ndim else exact[mask]).max(), 1.0)
    if got.ndim > mask.ndim:
        for k in range(got.shape[0]):
            assert np.abs(got[k][mask] - exact[k][mask]).max() <= rel * scale
            assert np.all(got[k][~mask] == 0.0)
    else:
        assert np.abs(got[mask] - exact[mask]).max() <= rel * scale
        assert np.all(got[~mask] == 0.0)


def test_gradient_exact_on_quadratics():
    blocks, levels = refined_layout()
    X, Y, Z = positions(blocks, levels, N_B)
    rng = np.random.default_rng(11)
    a, b = rng.normal(size=3), rng.normal(size=6)
    phi = (a[0] * X + a[1] * Y + a[2] * Z + b[0] * X * X + b[1] * Y * Y + b[2] * Z * Z
           + b[3] * X * Y + b[4] * Y * Z + b[5] * X * Z + 0.7)
    exact = np.stack([a[0] + 2 * b[0] * X + b[3] * Y + b[5] * Z,
                      a[1] + 2 * b[1] * Y + b[3] * X + b[4] * Z,
                      a[2] + 2 * b[2] * Z + b[4] * Y + b[5] * X])
    mask = operators.op_mask(blocks, levels, N_B)
    assert mask[levels == 1].any() and mask[levels == 0].any()
    # every cell of the refined blocks is evaluated, the interface cells among them
    inner = multires.residual_mask(blocks, levels, N_B)
    assert mask[levels == 1].all() and (mask & ~inner)[levels == 1].any()
    _check_on_mask(operators.apply(blocks, levels, phi, N_B, "gradient"), exact, mask)


def test_laplacian_exact_on_cubics_and_at_interfaces_on_quadratics():
    """Away from level boundaries the 7-point Laplacian is exact for cubics; on every evaluated
    cell (the interface cells take the parent's quadratic as neighbour) for quadratics."""
    blocks, levels = refined_layout()
    X, Y, Z = positions(blocks, levels, N_B)
    c = np.random.default_rng(12).normal(size=7)
    phi = (c[0] * X ** 3 + c[1] * X * X * Y + c[2] * X * Y * Z + c[3] * Z ** 3 + c[4] * Y * Y * Z
           + c[5] * X * X + c[6] * Y * Z)
    exact = 6 * c[0] * X + 2 * c[1] * Y + 6 * c[3] * Z + 2 * c[4] * Z + 2 * c[5]
    inner = multires.residual_mask(blocks, levels, N_B)
    got = operators.apply(blocks, levels, phi, N_B, "laplacian")
    assert np.abs(got[inner] - exact[inner]).max() <= 1e-12 * np.abs(exact[inner]).max()
    q = np.random.default_rng(15).normal(size=4)
    quad = q[0] * X * X + q[1] * Y * Z + q[2] * Z * Z + q[3] * X
    mask = operators.op_mask(blocks, levels, N_B)
    # rounding: the field reaches |quad| ~ 1e3 and the stencil scales it by h^-2 = 4
    _check_on_mask(operators.apply(blocks, levels, quad, N_B, "laplacian"),
                   np.full(X.shape, 2 * q[0] + 2 * q[2]), mask, rel=1e-14 * 4 * np.abs(quad).max())


def test_curl_exact_on_quadratic_fields():
    blocks, levels = refined_layout()
    X, Y, Z = positions(blocks, levels, N_B)
    k = np.random.default_rng(13).normal(size=(3, 4))
    # A_c = k_c0 + k_c1 q1 + k_c2 q2 + k_c3 q1 q2 with (q1, q2) the two other coordinates of c's
    # cyclic successors: A_x(y, z), A_y(z, x), A_z(x, y)
    A = np.stack([k[0, 0] + k[0, 1] * Y + k[0, 2] * Z + k[0, 3] * Y * Z,
                  k[1, 0] + k[1, 1] * Z + k[1, 2] * X + k[1, 3] * Z * X,
                  k[2, 0] + k[2, 1] * X + k[2, 2] * Y + k[2, 3] * X * Y])
    dAz_dy, dAy_dz = k[2, 2] + k[2, 3] * X, k[1, 1] + k[1, 3] * X
    dAx_dz, dAz_dx = k[0, 2] + k[0, 3] * Y, k[2, 1] + k[2, 3] * Y
    dAy_dx, dAx_dy = k[1, 2] + k[1, 3] * Z, k[0, 1] + k[0, 3] * Z
    exact = np.stack([dAz_dy - dAy_dz, dAx_dz - dAz_dx, dAy_dx - dAx_dy])
    mask = operators.op_mask(blocks, levels, N_B)
    _check_on_mask(operators.apply(blocks, levels, A, N_B, "curl"), exact, mask)


def test_interface_values_come_from_the_parent():
    """A field that is a different quadratic on each level: at a refinement interface the
    operators see the parent's polynomial outside the fine blocks, so the gradient of a fine
    interface cell mixes the two (not the fine quadratic's exact gradient); a planted zero ghost
    would give yet another value."""
    blocks, levels = refined_layout()
    X, Y, Z = positions(blocks, levels, N_B)
    fine = levels[:, None, None, None] == 1
    phi = np.where(fine, X * X, Y * Y + 1.0)          # the parent level holds y^2 + 1
    g = operators.apply(blocks, levels, phi, N_B, "gradient")
    i = int(np.nonzero(levels == 1)[0][0])            # child (2, 0, 2): its -x face is an interface
    h = 0.5
    x0, y0 = X[i, :, :, 0], Y[i, :, :, 0]
    # (u(x + h) - ghost) / 2h, the ghost the parent's quadratic y^2 + 1 at the ghost cell
    assert np.allclose(g[0, i, :, :, 0], ((x0 + h) ** 2 - (y0 * y0 + 1.0)) / (2 * h), rtol=0, atol=1e-11)
    assert np.allclose(g[0, i, :, :, 1:-1], 2 * X[i, :, :, 1:-1], rtol=0, atol=1e-11)


def test_curl_of_gradient_vanishes():
    blocks, levels = np.array([[0, 0, 0]], np.int32), np.array([0], np.int32)
    phi = np.random.default_rng(14).normal(size=(1, N_B, N_B, N_B))
    G = operators.apply(blocks, levels, phi, N_B, "gradient")
    C = operators.apply(blocks, levels, G, N_B, "curl")
    inner = (slice(None), slice(2, -2), slice(2, -2), slice(2, -2))
    assert np.abs(G).max() > 0.1
    for k in range(3):
        assert np.abs(C[k][inner]).max() <= 1e-13 * np.abs(G).max()


def test_laplacian_of_refined_solve_gives_source():
    blocks, levels, f, _ = gaussian_problem(N_B)
    mask = multires.residual_mask(blocks, levels, N_B)
    scale = np.abs(f).max()
    u = multires.solve(blocks, levels, f, N_B, 6, correction=True)
    lap = operators.apply(blocks, levels, u, N_B, "laplacian")
    assert np.abs(lap[mask] - f[mask]).max() <= 1e-12 * scale
    u0 = multires.solve(blocks, levels, f, N_B, 6, correction=False)
    lap0 = operators.apply(blocks, levels, u0, N_B, "laplacian")
    assert np.abs(lap0[mask] - f[mask]).max() > 1e-8 * scale
