"""Seeded synthetic inputs shared by the CPU oracle and the GPU library's tests.

This module only builds *problem data*: sparse SPD matrices in CSR form,
right-hand sides and random coefficient fields.  It holds none of the
smoother / multigrid / Krylov arithmetic, so it may be imported by both the
oracle and the GPU-side tests and benchmark without coupling them.

Ordering is lexicographic, row = i + nx*j + nx*ny*k, with Dirichlet unknowns
eliminated (only interior nodes are unknowns).  Within a row the column
indices are strictly increasing.

The workloads stand in for the paper's synthetic PDE test matrices (Poisson
3D 7-point, Section 4; the paper measures on no external dataset).
"""
from __future__ import annotations

from dataclasses import dataclass
from fractions import Fraction

import numpy as np

__all__ = [
    "CSR",
    "stencil_csr",
    "poisson2d_5pt",
    "poisson3d_7pt",
    "q1_27pt",
    "fv_diffusion",
    "gaussian_random_field",
    "rhs_uniform",
    "stack_block_diagonal",
    "config_problem",
    "SEED_RHS",
    "SEED_GRF",
    "SEED_MLP",
    "mlp_init",
    "config4_sigmas",
    "qdq_dense",
    "anisotropy2d_q1",
]

# Seed bases: b uses default_rng(SEED_RHS + config number), the Gaussian
# random field of problem p uses default_rng(SEED_GRF + p), the MLP initial
# weights use default_rng(SEED_MLP).
SEED_RHS = 1000
SEED_GRF = 2000
SEED_MLP = 3000


@dataclass
class CSR:
    """Host CSR matrix: int32 row_ptr/col, float64 val, plus grid shape."""

    n: int
    row_ptr: np.ndarray  # int64 during assembly, int32 when stored (nnz < 2**31)
    col: np.ndarray  # int32
    val: np.ndarray  # float64
    grid: tuple  # (nx, ny, nz)
    nbatch: int = 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def stencil_csr(grid, offsets, values, planes_per_chunk=None):
    """Assemble a CSR matrix from a stencil on an (nx, ny, nz) interior grid.

    ``offsets`` is a list of (dx, dy, dz); ``values[m]`` is either a scalar or
    an array of shape (nz, ny, nx) giving the coefficient that row (i,j,k)
    places on its neighbour (i+dx, j+dy, k+dz).  Neighbours outside the grid
    are dropped (Dirichlet elimination).  Entries are stored even when their
    value is exactly zero (the stencil pattern, not the values, fixes nnz).
    Rows are built a few z-planes at a time as dense (rows x stencil) blocks
    compressed by the validity mask, which keeps memory bounded.
    """
    nx, ny, nz = grid
    n = nx * ny * nz
    order = sorted(range(len(offsets)), key=lambda m: (offsets[m][2], offsets[m][1], offsets[m][0]))
    offs = np.array([offsets[m] for m in order], dtype=np.int64)
    vals = [values[m] for m in order]
    M = len(order)
    vx = (np.arange(nx)[:, None] + offs[None, :, 0] >= 0) & (np.arange(nx)[:, None] + offs[None, :, 0] < nx)
    vy = (np.arange(ny)[:, None] + offs[None, :, 1] >= 0) & (np.arange(ny)[:, None] + offs[None, :, 1] < ny)
    vz = (np.arange(nz)[:, None] + offs[None, :, 2] >= 0) & (np.arange(nz)[:, None] + offs[None, :, 2] < nz)
    plane_cnt = (vy[:, None, :] & vx[None, :, :])  # (ny, nx, M)
    counts = np.empty(n, dtype=np.int64)
    for k in range(nz):
        counts[k * nx * ny:(k + 1) * nx * ny] = (plane_cnt & vz[k][None, None, :]).sum(axis=2).ravel()
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    if nnz >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    delta = (offs[:, 0] + nx * offs[:, 1] + nx * ny * offs[:, 2]).astype(np.int32)
    kc = planes_per_chunk or max(1, (1 << 20) // (nx * ny))
    rows_max = min(nz, kc) * nx * ny
    # chunk buffers reused across chunks (first-touch allocation dominates otherwise)
    cols = np.empty((rows_max, M), dtype=np.int32)
    block = np.empty((rows_max, M), dtype=np.float64)
    mask = np.empty((rows_max, M), dtype=bool)
    base = np.arange(rows_max, dtype=np.int32)
    all_scalar = all(np.isscalar(v) for v in vals)
    scalar_row = np.array([float(v) for v in vals]) if all_scalar else None
    for k0 in range(0, nz, kc):
        k1 = min(nz, k0 + kc)
        r0, r1 = k0 * nx * ny, k1 * nx * ny
        m_ = mask[:r1 - r0]
        np.logical_and(plane_cnt[None, :, :, :], vz[k0:k1, None, None, :], out=m_.reshape(k1 - k0, ny, nx, M))
        c_ = cols[:r1 - r0]
        np.add(base[:r1 - r0, None], np.int32(r0) + delta[None, :], out=c_)
        col[row_ptr[r0]:row_ptr[r1]] = c_[m_]
        b_ = block[:r1 - r0]
        if all_scalar:
            b_[...] = scalar_row[None, :]
        else:
            for m, v in enumerate(vals):
                b_[:, m] = v if np.isscalar(v) else np.asarray(v, dtype=np.float64)[k0:k1].ravel()
        val[row_ptr[r0]:row_ptr[r1]] = b_[m_]
    return CSR(n=n, row_ptr=row_ptr.astype(np.int32), col=col, val=val, grid=(nx, ny, nz))


def poisson2d_5pt(nx: int, ny: int) -> CSR:
    """2D 5-point Laplacian, diagonal 4, neighbours -1, on an nx*ny interior grid."""
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0)]
    vals = [4.0, -1.0, -1.0, -1.0, -1.0]
    return stencil_csr((nx, ny, 1), offs, vals)


def poisson3d_7pt(nx: int, ny: int | None = None, nz: int | None = None) -> CSR:
    """3D 7-point Laplacian, diagonal 6, neighbours -1."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    offs = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    vals = [6.0, -1.0, -1.0, -1.0, -1.0, -1.0, -1.0]
    return stencil_csr((nx, ny, nz), offs, vals)


def q1_27pt(nx: int, ny: int | None = None, nz: int | None = None, store_zeros: bool = True) -> CSR:
    """3D trilinear (Q1) finite-element Laplacian on a uniform hexahedral mesh.

    Stencil (mesh-size factor dropped): centre 8/3, the 6 face neighbours 0
    (stored explicitly, they belong to the 27-point pattern), the 12 edge
    neighbours -1/6, the 8 corner neighbours -1/12.  Values are taken from
    exact rationals and rounded once to float64.  store_zeros=False leaves the
    six zero face entries out (the same operator with a 21-point pattern, what
    a caller gets by eliminating stored zeros).
    """
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    offs, vals = [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = abs(dx) + abs(dy) + abs(dz)
                v = {0: Fraction(8, 3), 1: Fraction(0), 2: Fraction(-1, 6), 3: Fraction(-1, 12)}[d]
                if v == 0 and not store_zeros:
                    continue
                offs.append((dx, dy, dz))
                vals.append(float(v))
    return stencil_csr((nx, ny, nz), offs, vals)


def fv_diffusion(kappa: np.ndarray) -> CSR:
    """7-point cell-centred finite-volume discretisation of -div(kappa grad u).

    ``kappa`` has shape (nz, ny, nx).  Interior face transmissibility is the
    harmonic mean 2*k_i*k_j/(k_i+k_j); a boundary face (homogeneous Dirichlet
    at the face, half a cell away) contributes 2*k_i to the diagonal.  Unit
    mesh size.  The diagonal is the sum of the row's six face
    transmissibilities, so the matrix is SPD.
    """
    kappa = np.asarray(kappa, dtype=np.float64)
    nz, ny, nx = kappa.shape
    def harm(a, b):
        return 2.0 * a * b / (a + b)
    diag = np.zeros_like(kappa)
    off = {}
    for axis, (dx, dy, dz) in zip((2, 1, 0), ((1, 0, 0), (0, 1, 0), (0, 0, 1))):
        # transmissibility between cell c and c+e along this axis
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[axis] = slice(0, -1)
        sl_hi[axis] = slice(1, None)
        t = harm(kappa[tuple(sl_lo)], kappa[tuple(sl_hi)])
        plus = np.zeros_like(kappa)
        minus = np.zeros_like(kappa)
        plus[tuple(sl_lo)] = t   # row c, neighbour c+e
        minus[tuple(sl_hi)] = t  # row c+e, neighbour c
        off[(dx, dy, dz)] = -plus
        off[(-dx, -dy, -dz)] = -minus
        # diagonal: interior faces plus Dirichlet boundary faces
        bnd = np.zeros_like(kappa)
        first = [slice(None)] * 3
        last = [slice(None)] * 3
        first[axis] = 0
        last[axis] = -1
        bnd[tuple(first)] += 2.0 * kappa[tuple(first)]
        bnd[tuple(last)] += 2.0 * kappa[tuple(last)]
        diag += plus + minus + bnd
    offs = [(0, 0, 0)] + list(off.keys())
    vals = [diag] + [off[o] for o in off]
    return stencil_csr((nx, ny, nz), offs, vals)


def gaussian_random_field(shape, ell: float, seed: int) -> np.ndarray:
    """Stationary Gaussian random field on a periodic box, squared-exponential covariance.

    g = real(IFFT(sqrt(S(k)) * FFT(w))) with w i.i.d. N(0,1) from
    ``numpy.random.default_rng(seed)`` and S(k) = exp(-ell^2 |k|^2 / 2) the
    (unnormalised) spectral density of exp(-r^2 / (2 ell^2)).  The result is
    standardised to zero sample mean and unit sample standard deviation.
    ``shape`` is (nz, ny, nx); ``ell`` is in cells.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(shape)
    nz, ny, nx = shape
    kz = 2 * np.pi * np.fft.fftfreq(nz)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    kx = 2 * np.pi * np.fft.rfftfreq(nx)
    k2 = kz[:, None, None] ** 2 + ky[None, :, None] ** 2 + kx[None, None, :] ** 2
    amp = np.exp(-0.25 * ell * ell * k2)  # sqrt(S)
    g = np.fft.irfftn(np.fft.rfftn(w) * amp, s=shape, axes=(0, 1, 2))
    g -= g.mean()
    g /= g.std()
    return g


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """b ~ U(-1, 1)^n in float64 from ``numpy.random.default_rng(seed)``."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def stack_block_diagonal(mats) -> CSR:
    """Stack equally shaped grid problems along z into one block-diagonal matrix."""
    mats = list(mats)
    g = mats[0].grid
    n0 = mats[0].n
    for m in mats:
        if m.grid != g or m.n != n0:
            raise ValueError("all blocks must share one grid")
    nnzs = [m.nnz for m in mats]
    row_ptr = np.zeros(n0 * len(mats) + 1, dtype=np.int64)
    col = np.empty(sum(nnzs), dtype=np.int32)
    val = np.empty(sum(nnzs), dtype=np.float64)
    off = 0
    for b, m in enumerate(mats):
        row_ptr[b * n0 + 1:(b + 1) * n0 + 1] = m.row_ptr[1:].astype(np.int64) + off
        col[off:off + m.nnz] = m.col + b * n0
        val[off:off + m.nnz] = m.val
        off += m.nnz
    return CSR(n=n0 * len(mats), row_ptr=row_ptr.astype(np.int32), col=col, val=val,
               grid=(g[0], g[1], g[2] * len(mats)), nbatch=len(mats))


def config_problem(cfg: int, size: int | None = None):
    """Matrix and right-hand side of workload ``cfg`` (1..5), optionally at a smaller edge.

    1: 2D 5-point Poisson, 64x64 interior.
    2: 3D 7-point Poisson, 128^3.
    3: 3D FV diffusion, kappa = exp(g), g a GRF with correlation length 8 cells, sigma = 1, 256^3.
    4: 32 stacked 3D FV diffusion problems at 64^3, sigma cycling over (0.5, 1, 2).
    5: 3D 27-point Q1 Laplacian, 320^3.
    Returns (CSR, b, meta dict).
    """
    if cfg == 1:
        s = 64 if size is None else size
        A = poisson2d_5pt(s, s)
        meta = {"dim": 2}
    elif cfg == 2:
        s = 128 if size is None else size
        A = poisson3d_7pt(s)
        meta = {"dim": 3}
    elif cfg == 3:
        s = 256 if size is None else size
        g = gaussian_random_field((s, s, s), 8.0, SEED_GRF + 0)
        A = fv_diffusion(np.exp(1.0 * g))
        meta = {"dim": 3, "sigma": 1.0}
    elif cfg == 4:
        s = 64 if size is None else size
        sig = (0.5, 1.0, 2.0)
        probs = []
        sigmas = []
        for p in range(32):
            g = gaussian_random_field((s, s, s), 8.0, SEED_GRF + p)
            probs.append(fv_diffusion(np.exp(sig[p % 3] * g)))
            sigmas.append(sig[p % 3])
        A = stack_block_diagonal(probs)
        meta = {"dim": 3, "sigmas": sigmas}
    elif cfg == 5:
        s = 320 if size is None else size
        A = q1_27pt(s)
        meta = {"dim": 3}
    else:
        raise ValueError(cfg)
    b = rhs_uniform(A.n, SEED_RHS + cfg)
    return A, b, meta


def config4_sigmas(nprob=32):
    """sigma of stacked problem p in the learned-weights workload: cycles over (0.5, 1, 2)."""
    return [(0.5, 1.0, 2.0)[p % 3] for p in range(nprob)]


def mlp_init(seed: int = SEED_MLP):
    """Initial parameters of the 8-64-64-6 network, float64 vector of 5126 entries laid out as
    W1[64][8], b1[64], W2[64][64], b2[64], W3[6][64], b3[6]: weights ~ U(-1/sqrt(fan_in),
    1/sqrt(fan_in)) drawn in that order from default_rng(seed), biases 0."""
    rng = np.random.default_rng(seed)
    parts = []
    for shape, is_w in (((64, 8), True), ((64,), False), ((64, 64), True), ((64,), False),
                        ((6, 64), True), ((6,), False)):
        if is_w:
            bound = 1.0 / np.sqrt(shape[1])
            parts.append(rng.uniform(-bound, bound, shape).ravel())
        else:
            parts.append(np.zeros(shape))
    return np.concatenate(parts)


def qdq_dense(N: int, spectrum: str):
    """Dense SPD test matrix A = Q D Q^T of the polynomial-preconditioning experiment
    (the remark after Fig. boundcomparison, Fig. better-than-optimal).

    Q holds the orthonormal eigenvectors of the 1D second-difference matrix
    tridiag(-1, 2, -1) of order N, the discrete sines
    Q[i, j] = sqrt(2/(N+1)) sin((i+1)(j+1) pi/(N+1)).  D (N even) is one of
      'equispaced': N points equally spaced in [1/N, 1];
      'clustered':  1 - logspace(-8, -1, N/2) followed by logspace(-8, -1, N/2),
                    eigenvalues accumulating at both ends of (0, 1);
      'gap':        logspace(-8, -1, N/2) followed by N/2 points logarithmically
                    spaced from 10 down to pi (the MATLAB meaning of logspace(1, pi, m)).
    The right-hand side is b = A 1.  Returns (CSR with full rows, b, d).
    """
    if N < 2 or N % 2:
        raise ValueError("N must be even and >= 2")
    m = N // 2
    if spectrum == "equispaced":
        d = np.linspace(1.0 / N, 1.0, N)
    elif spectrum == "clustered":
        lo = np.logspace(-8, -1, m)
        d = np.concatenate([1.0 - lo, lo])
    elif spectrum == "gap":
        d = np.concatenate([np.logspace(-8, -1, m), 10.0 ** np.linspace(1.0, np.log10(np.pi), m)])
    else:
        raise ValueError(spectrum)
    idx = np.arange(1, N + 1, dtype=np.float64)
    Q = np.sqrt(2.0 / (N + 1)) * np.sin(np.outer(idx, idx) * np.pi / (N + 1))
    A = (Q * d[None, :]) @ Q.T
    A = 0.5 * (A + A.T)  # exactly symmetric
    b = A @ np.ones(N)
    row_ptr = (np.arange(N + 1, dtype=np.int64) * N).astype(np.int32)
    col = np.tile(np.arange(N, dtype=np.int32), N)
    return CSR(n=N, row_ptr=row_ptr, col=col, val=A.ravel().copy(), grid=(N, 1, 1)), b, d


def _q1_element_2d(kxx: float, kxy: float, kyy: float) -> np.ndarray:
    """Stiffness of one bilinear square element for the constant tensor K (mesh-size free in 2D),
    exact by 2x2 Gauss quadrature.  Local node (a, b) = (x offset, y offset) has index a + 2b."""
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    Ke = np.zeros((4, 4))
    K = np.array([[kxx, kxy], [kxy, kyy]])
    for xi in g:
        for eta in g:
            grads = []
            for b_ in (0, 1):
                for a_ in (0, 1):
                    fx = xi if a_ else 1.0 - xi
                    fy = eta if b_ else 1.0 - eta
                    dfx = 1.0 if a_ else -1.0
                    dfy = 1.0 if b_ else -1.0
                    grads.append((dfx * fy, fx * dfy))
            G = np.array(grads)  # (4, 2)
            Ke += 0.25 * G @ K @ G.T
    return 0.5 * (Ke + Ke.T)  # exactly symmetric, so the assembled matrix is too


def anisotropy2d_q1(N: int, eps: float = 100.0, theta: float = np.pi / 6):
    """Anisotropic 2D thermal problem of Section 4 ("Anisotropy 2D"), Q1 finite elements.

    Domain [-1, 1]^2 split into N x N square elements; conductivity
    K = R(theta) diag(1, eps) R(theta)^T; homogeneous Dirichlet condition on the
    face y = -1 (those nodes are eliminated), natural (Neumann) conditions on the
    other three faces; load f(x, y) = exp(-100 (x^2 + y^2)) integrated against
    the basis functions with 2x2 Gauss points per element.
    Unknowns: the (N+1) x N nodes with y > -1, ordered i + (N+1) j (x fastest),
    so grid = (N+1, N, 1).  Each row has the 9-point pattern of its node.
    Returns (CSR, b).
    """
    c, s_ = np.cos(theta), np.sin(theta)
    kxx = c * c + eps * s_ * s_
    kyy = s_ * s_ + eps * c * c
    kxy = (1.0 - eps) * s_ * c
    Ke = _q1_element_2d(kxx, kxy, kyy)
    nxn, nyn = N + 1, N + 1  # all nodes, including y = -1
    I = np.arange(nxn)[None, :]
    J = np.arange(nyn)[:, None]
    offs, vals = [], []
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            v = np.zeros((nyn, nxn))
            for ea in (-1, 0):
                for eb in (-1, 0):
                    a_, b_ = -ea, -eb  # local position of the row node in element (i+ea, j+eb)
                    a2, b2 = a_ + dx, b_ + dy
                    if not (0 <= a2 <= 1 and 0 <= b2 <= 1):
                        continue
                    ok = (I + ea >= 0) & (I + ea <= N - 1) & (J + eb >= 0) & (J + eb <= N - 1)
                    v += np.where(ok, Ke[a_ + 2 * b_, a2 + 2 * b2], 0.0)
            offs.append((dx, dy, 0))
            vals.append(v[1:][None, :, :])  # drop the Dirichlet row y = -1
    A = stencil_csr((nxn, N, 1), offs, vals)
    # load vector
    h = 2.0 / N
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    x0 = -1.0 + h * np.arange(N)
    F = np.zeros((nyn, nxn))
    for xi in g:
        for eta in g:
            fq = np.exp(-100.0 * ((x0[None, :] + h * xi) ** 2 + (x0[:, None] + h * eta) ** 2)) * (h * h / 4.0)
            for b_ in (0, 1):
                for a_ in (0, 1):
                    phi = (xi if a_ else 1.0 - xi) * (eta if b_ else 1.0 - eta)
                    F[b_:b_ + N, a_:a_ + N] += phi * fq
    b = F[1:].ravel().copy()
    return A, b
