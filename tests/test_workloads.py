"""Pins of the seeded input generators against closed forms that do not share their assembly.

* 7-point and 27-point Q1 operators: the Kronecker-sum forms of the 1D second difference K and
  the 1D Q1 mass matrix M (Dirichlet elimination keeps them tridiagonal of order n), the pattern
  sizes 7n^3 - 6n^2 and (3n - 2)^3, and the exactly stored zero face entries.
* FV diffusion: with a constant conductivity c it is c times the 7-point Laplacian plus c per
  boundary face of a cell (a boundary face weighs 2c, an interior face c); for any conductivity
  it is symmetric with row sums equal to the boundary terms.
* The bilinear element for K = I is the textbook one; the anisotropic problem at theta = 0 is
  M_y (x) K_x + eps K_y (x) M_x with natural ends in x and at y = 1 and the node row y = -1
  eliminated; for any angle it is symmetric positive definite, its rows away from the
  Dirichlet face sum to zero, and the load is mirror-symmetric in x.
* The random field is standardised; the Q D Q^T matrices have exactly the requested spectra.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W


def _tri(n, d, o, d_end=None):
    main = np.full(n, d, dtype=np.float64)
    if d_end is not None:
        main[0] = main[-1] = d_end
    return sp.diags([np.full(n - 1, o), main, np.full(n - 1, o)], [-1, 0, 1], format="csr")


@pytest.mark.parametrize("dims", [(5, 4, 3), (6, 6, 6)])
def test_7pt_is_kronecker_sum(dims):
    nx, ny, nz = dims
    A = W.poisson3d_7pt(nx, ny, nz)
    K = [_tri(m, 2.0, -1.0) for m in dims]
    I = [sp.identity(m, format="csr") for m in dims]
    ref = sp.kron(I[2], sp.kron(I[1], K[0])) + sp.kron(I[2], sp.kron(K[1], I[0])) + sp.kron(K[2], sp.kron(I[1], I[0]))
    assert abs(A.to_scipy() - ref).max() == 0.0
    if nx == ny == nz:
        assert A.nnz == 7 * nx**3 - 6 * nx**2


@pytest.mark.parametrize("n", [3, 5])
def test_q1_27pt_is_kronecker_sum_of_stiffness_and_mass(n):
    A = W.q1_27pt(n)
    K = _tri(n, 2.0, -1.0)
    M = _tri(n, 4.0 / 6.0, 1.0 / 6.0)
    ref = sp.kron(M, sp.kron(M, K)) + sp.kron(M, sp.kron(K, M)) + sp.kron(K, sp.kron(M, M))
    As = A.to_scipy()
    assert np.abs(As.toarray() - ref.toarray()).max() <= 1e-15
    assert A.nnz == (3 * n - 2) ** 3
    # the face neighbours are stored although they are zero
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    face = np.isin(np.abs(A.col.astype(np.int64) - rows), [1, n, n * n])
    assert np.all(A.val[face] == 0.0) and face.sum() > 0


@pytest.mark.parametrize("n", [3, 6])
def test_q1_without_stored_zeros_is_the_same_operator(n):
    A, B = W.q1_27pt(n), W.q1_27pt(n, store_zeros=False)
    S = A.to_scipy().copy()
    S.eliminate_zeros()
    assert np.array_equal(S.indptr, B.row_ptr) and np.array_equal(S.indices, B.col)
    assert np.array_equal(S.data, B.val)
    # 27 minus the six faces per interior row; in all, the face pairs of the grid are gone
    faces = 3 * (n - 1) * n * n
    assert B.nnz == A.nnz - 2 * faces


def test_fv_constant_conductivity_closed_form():
    shape = (4, 5, 6)  # (nz, ny, nx)
    c = 2.5
    A = W.fv_diffusion(np.full(shape, c)).to_scipy()
    nz, ny, nx = shape
    L = W.poisson3d_7pt(nx, ny, nz).to_scipy()
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    faces = ((x == 0).astype(int) + (x == nx - 1) + (y == 0) + (y == ny - 1) + (z == 0) + (z == nz - 1)).ravel()
    ref = c * L + sp.diags(c * faces.astype(np.float64))
    assert abs(A - ref).max() <= 1e-14


def test_fv_symmetric_with_boundary_row_sums():
    kappa = np.exp(1.5 * W.gaussian_random_field((5, 6, 7), 2.0, 11))
    A = W.fv_diffusion(kappa).to_scipy()
    assert abs(A - A.T).max() == 0.0
    nz, ny, nx = kappa.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    faces = ((x == 0).astype(int) + (x == nx - 1) + (y == 0) + (y == ny - 1) + (z == 0) + (z == nz - 1)).ravel()
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.allclose(rs, 2.0 * kappa.ravel() * faces, rtol=1e-13, atol=1e-13 * kappa.max())
    # off-diagonal entries lie between the two conductivities (a harmonic mean does)
    Ac = A.tocoo()
    off = Ac.row != Ac.col
    ki, kj = kappa.ravel()[Ac.row[off]], kappa.ravel()[Ac.col[off]]
    t = -Ac.data[off]
    assert np.all(t >= np.minimum(ki, kj) * (1 - 1e-14)) and np.all(t <= np.maximum(ki, kj) * (1 + 1e-14))


def test_gaussian_random_field_is_standardised_and_seeded():
    g = W.gaussian_random_field((8, 10, 12), 3.0, 5)
    assert abs(g.mean()) <= 1e-14 and abs(g.std() - 1.0) <= 1e-13
    assert np.array_equal(g, W.gaussian_random_field((8, 10, 12), 3.0, 5))
    assert not np.array_equal(g, W.gaussian_random_field((8, 10, 12), 3.0, 6))
    # a longer correlation length gives a smoother field (smaller mean squared increment)
    rough = W.gaussian_random_field((16, 16, 16), 1.0, 5)
    smooth = W.gaussian_random_field((16, 16, 16), 4.0, 5)
    assert np.mean(np.diff(smooth, axis=2) ** 2) < np.mean(np.diff(rough, axis=2) ** 2)


def test_bilinear_element_for_identity_conductivity():
    Ke = W._q1_element_2d(1.0, 0.0, 1.0)
    # local nodes (0,0), (1,0), (0,1), (1,1): edge neighbours -1/6, opposite corner -1/3
    ref = np.array([[4, -1, -1, -2], [-1, 4, -2, -1], [-1, -2, 4, -1], [-2, -1, -1, 4]]) / 6.0
    assert np.abs(Ke - ref).max() <= 1e-15


def test_anisotropy_at_zero_angle_is_kronecker_form():
    N, eps = 6, 100.0
    A, _ = W.anisotropy2d_q1(N, eps=eps, theta=0.0)
    nxn = N + 1
    Kx = _tri(nxn, 2.0, -1.0, d_end=1.0)
    Mx = _tri(nxn, 4.0 / 6.0, 1.0 / 6.0, d_end=2.0 / 6.0)
    # y: nodes y_1 .. y_N (y_0 = -1 eliminated), natural end at y_N = 1
    Ky = _tri(N, 2.0, -1.0)
    My = _tri(N, 4.0 / 6.0, 1.0 / 6.0)
    Ky = Ky.tolil()
    My = My.tolil()
    Ky[N - 1, N - 1] = 1.0
    My[N - 1, N - 1] = 2.0 / 6.0
    ref = sp.kron(My.tocsr(), Kx) + eps * sp.kron(Ky.tocsr(), Mx)
    assert A.grid == (nxn, N, 1)
    assert np.abs(A.to_scipy().toarray() - ref.toarray()).max() <= 1e-12 * eps


def test_anisotropy_rotated_is_spd_with_zero_row_sums_and_symmetric_load():
    N = 8
    A, b = W.anisotropy2d_q1(N)
    As = A.to_scipy()
    assert abs(As - As.T).max() <= 1e-13
    assert np.linalg.eigvalsh(As.toarray()).min() > 0
    rs = np.asarray(As.sum(axis=1)).ravel().reshape(N, N + 1)
    assert np.abs(rs[1:]).max() <= 1e-12  # rows not adjacent to the eliminated face y = -1
    assert np.abs(rs[0]).max() > 1e-3
    B = b.reshape(N, N + 1)
    assert np.abs(B - B[:, ::-1]).max() <= 1e-15 * np.abs(B).max() + 1e-300
    assert np.all(B > 0)


@pytest.mark.parametrize("spectrum", ["equispaced", "clustered", "gap"])
def test_qdq_has_the_requested_spectrum(spectrum):
    N = 32
    A, b, d = W.qdq_dense(N, spectrum)
    Ad = A.val.reshape(N, N)
    ev = np.linalg.eigvalsh(Ad)
    assert np.allclose(np.sort(ev), np.sort(d), rtol=1e-12, atol=1e-14)
    assert np.allclose(b, Ad @ np.ones(N), rtol=0, atol=1e-14)
    if spectrum == "gap":
        assert np.isclose(d.max(), 10.0) and np.isclose(d[N // 2:].min(), np.pi)
