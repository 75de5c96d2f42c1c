"""Oracle: lattice geometry, gamma matrices, dense Wilson matrix, free-field
closed forms (test infrastructure only).

The paper estimates Tr(Theta M^-1) for the Wilson-Dirac matrix M with hopping
parameter kappa (Sec. 1 eq. 1, Sec. 4) but never writes M out.  Reading used
throughout the oracle (and stated in the design notes):

    (M psi)(x) = psi(x) - kappa sum_mu [ (1 - gamma_mu) U_mu(x) psi(x+mu)
                                       + (1 + gamma_mu) U_mu(x-mu)^H psi(x-mu) ]

DeGrand-Rossi gammas, periodic space, antiperiodic time (a hop across the time
boundary picks up -1).  Component index c = (s*4 + spin)*3 + colour with
s = x + Lx*(y + Ly*(z + Lz*t)).

Pins (tests/test_oracle_lattice.py): gamma algebra; the momentum-space symbol
of the free operator on plane waves; the free-field closed-form trace; kappa=0;
gamma5-hermiticity; gauge covariance; matrix-free C operator == dense matrix.
"""
import numpy as np

# DeGrand-Rossi basis, mu = 0..3 = x, y, z, t.
GAMMA = np.array([
    [[0, 0, 0, 1j], [0, 0, 1j, 0], [0, -1j, 0, 0], [-1j, 0, 0, 0]],
    [[0, 0, 0, -1], [0, 0, 1, 0], [0, 1, 0, 0], [-1, 0, 0, 0]],
    [[0, 0, 1j, 0], [0, 0, 0, -1j], [-1j, 0, 0, 0], [0, 1j, 0, 0]],
    [[0, 0, 1, 0], [0, 0, 0, 1], [1, 0, 0, 0], [0, 1, 0, 0]],
], dtype=np.complex128)
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]


def volume(dims):
    return int(dims[0]) * int(dims[1]) * int(dims[2]) * int(dims[3])


def coords(dims):
    """Coordinates (V, 4) of every site in canonical order (x fastest)."""
    V = volume(dims)
    s = np.arange(V)
    out = np.empty((V, 4), dtype=np.int64)
    for mu in range(4):
        out[:, mu] = s % dims[mu]
        s = s // dims[mu]
    return out


def site_index(c, dims):
    c = np.asarray(c)
    return c[..., 0] + dims[0] * (c[..., 1] + dims[1] * (c[..., 2] + dims[2] * c[..., 3]))


def neighbour(dims, mu, step):
    """Site index of x + step*mu for every site x, and the boundary sign for an
    antiperiodic time direction."""
    c = coords(dims)
    cn = c.copy()
    cn[:, mu] = (c[:, mu] + step) % dims[mu]
    if mu == 3:
        crossed = (c[:, 3] == dims[3] - 1) if step > 0 else (c[:, 3] == 0)
    else:
        crossed = np.zeros(len(c), dtype=bool)
    return site_index(cn, dims), crossed


def theta_matrix(theta):
    """Spin matrix of the inserted operator: 'I' or 'g5'."""
    return np.eye(4, dtype=np.complex128) if theta in ("I", 0) else GAMMA5.copy()


def dense_wilson(dims, kappa, U, t_antiperiodic=True, dagger=False):
    """Dense n x n Wilson matrix (n = 12 V), built from Kronecker blocks.

    Only for small lattices (n <= ~6000).  Hops that land on the same site
    (L = 1 or 2) are accumulated, never overwritten.
    """
    V = volume(dims)
    n = 12 * V
    M = np.zeros((V, 4, 3, V, 4, 3), dtype=np.complex128)
    g = -1.0 if dagger else 1.0
    eye4 = np.eye(4)
    for mu in range(4):
        fwd, crossed_f = neighbour(dims, mu, +1)
        bwd, crossed_b = neighbour(dims, mu, -1)
        Pm = eye4 - g * GAMMA[mu]
        Pp = eye4 + g * GAMMA[mu]
        for s in range(V):
            sf = (-1.0 if (t_antiperiodic and crossed_f[s]) else 1.0)
            sb = (-1.0 if (t_antiperiodic and crossed_b[s]) else 1.0)
            # (1 - g gamma) (x) U_mu(x)            acting on psi(x+mu)
            M[s, :, :, fwd[s], :, :] += -kappa * sf * np.einsum("ab,ij->aibj", Pm, U[s, mu])
            # (1 + g gamma) (x) U_mu(x-mu)^H       acting on psi(x-mu)
            M[s, :, :, bwd[s], :, :] += -kappa * sb * np.einsum(
                "ab,ij->aibj", Pp, np.conj(U[bwd[s], mu]).T)
    M = M.reshape(n, n)
    M += np.eye(n)
    return M


def spin_op(vec, S):
    """Apply a 4x4 spin matrix to canonical vectors (..., n)."""
    v = vec.reshape(vec.shape[:-1] + (-1, 4, 3))
    return np.einsum("ab,...sbc->...sac", S, v).reshape(vec.shape)


def free_momenta(dims, t_antiperiodic=True):
    """All lattice momenta (V, 4): 2 pi n / L in space, (2n+1) pi / T in time."""
    axes = []
    for mu in range(4):
        k = np.arange(dims[mu])
        if mu == 3 and t_antiperiodic:
            axes.append((2 * k + 1) * np.pi / dims[mu])
        else:
            axes.append(2 * k * np.pi / dims[mu])
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.reshape(-1) for g in grid], axis=-1)


def free_symbol(p, kappa):
    """Momentum-space free Wilson operator a + i sum_mu b_mu gamma_mu,
    a = 1 - 2 kappa sum cos p_mu, b_mu = 2 kappa sin p_mu (4x4 spin matrix)."""
    a = 1 - 2 * kappa * np.sum(np.cos(p))
    return a * np.eye(4) + 1j * sum(2 * kappa * np.sin(p[mu]) * GAMMA[mu] for mu in range(4))


def free_trace_inverse(dims, kappa, t_antiperiodic=True):
    """Closed form Tr M^-1 = sum_p 12 a / (a^2 + |b|^2) for unit links."""
    p = free_momenta(dims, t_antiperiodic)
    a = 1 - 2 * kappa * np.cos(p).sum(axis=1)
    b2 = (2 * kappa * np.sin(p)) ** 2
    return float(np.sum(12 * a / (a * a + b2.sum(axis=1))))


def free_eigenvalues(dims, kappa, t_antiperiodic=True):
    """Closed-form spectrum of the free operator: a +- i|b|, each 6-fold."""
    p = free_momenta(dims, t_antiperiodic)
    a = 1 - 2 * kappa * np.cos(p).sum(axis=1)
    b = np.sqrt(((2 * kappa * np.sin(p)) ** 2).sum(axis=1))
    lam = np.concatenate([a + 1j * b, a - 1j * b])
    return np.repeat(lam, 6)


def plane_wave(dims, p, chi):
    """psi(x) = exp(i p.x) chi, chi a (4, 3) spin-colour vector; canonical layout."""
    c = coords(dims)
    phase = np.exp(1j * (c @ p))
    return (phase[:, None, None] * chi[None]).reshape(-1)


def gauge_rotate(U, g, dims):
    """U'_mu(x) = g(x) U_mu(x) g(x+mu)^H."""
    out = np.empty_like(U)
    for mu in range(4):
        fwd, _ = neighbour(dims, mu, +1)
        out[:, mu] = g @ U[:, mu] @ np.conj(np.transpose(g[fwd], (0, 2, 1)))
    return out


def colour_rotate(vec, g):
    """(G psi)(x) = g(x) psi(x) on canonical vectors (..., n)."""
    v = vec.reshape(vec.shape[:-1] + (-1, 4, 3))
    return np.einsum("sij,...saj->...sai", g, v).reshape(vec.shape)
