"""Seeded synthetic inputs: SU(3) gauge links.

This module is the only code that both the GPU path and the FP64 oracle use,
and it holds none of the method's arithmetic: it only manufactures the gauge
field the Wilson-Dirac matrix is built from.  The paper measures on quenched
beta = 6.0 configurations (Sec. 4, Sec. 8) that are not available here; these
fields stand in for them with the same lattice shapes.

Recipe: for every link (site, mu) draw a_1..a_8 ~ N(0, 1) from NumPy's PCG64
generator seeded with ``seed`` (in site-major, mu, k order), form the Hermitian
H = sum_k a_k lambda_k with the Gell-Mann matrices (tr lambda_a lambda_b =
2 delta_ab), exponentiate U = exp(i eps H) through the eigendecomposition of H,
and re-unitarise: Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1),
which makes det U = 1 to rounding.

Canonical link layout: complex128 array [V][4][3][3], site
s = x + Lx*(y + Ly*(z + Lz*t)), mu = 0..3 = x, y, z, t, U[s, mu, a, b] is
row a, column b of U_mu(s).
"""
import numpy as np


def gell_mann():
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1] = -1j
    l[1][1, 0] = 1j
    l[2][0, 0] = 1
    l[2][1, 1] = -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2] = -1j
    l[4][2, 0] = 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2] = -1j
    l[6][2, 1] = 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def volume(dims):
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


def reunitarise(U):
    """Project (..., 3, 3) matrices back onto SU(3) by row Gram-Schmidt."""
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def gauge_links(dims, eps, seed, chunk=1 << 16):
    """Random SU(3) links U = exp(i eps H) (see module docstring)."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    lam = gell_mann()
    out = np.empty((V, 4, 3, 3), dtype=np.complex128)
    flat = out.reshape(V * 4, 3, 3)
    total = V * 4
    for lo in range(0, total, chunk):
        hi = min(total, lo + chunk)
        a = rng.standard_normal((hi - lo, 8))
        H = np.einsum("nk,kab->nab", a, lam)
        w, Q = np.linalg.eigh(H)
        E = np.exp(1j * eps * w)
        U = np.einsum("nab,nb,ncb->nac", Q, E, np.conj(Q))
        flat[lo:hi] = reunitarise(U)
    return out


def unit_links(dims):
    """Free field: every link is the identity."""
    V = volume(dims)
    out = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    out[:, :, 0, 0] = out[:, :, 1, 1] = out[:, :, 2, 2] = 1
    return out


def random_gauge_transform(dims, seed):
    """Random SU(3) matrices g(x), one per site, shape (V, 3, 3) (for covariance tests)."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    A = rng.standard_normal((V, 3, 3)) + 1j * rng.standard_normal((V, 3, 3))
    Q, R = np.linalg.qr(A)
    Q = Q * (np.diagonal(R, axis1=-2, axis2=-1) / np.abs(np.diagonal(R, axis1=-2, axis2=-1)))[:, None, :]
    return reunitarise(Q)
