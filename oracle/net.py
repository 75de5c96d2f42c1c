"""Oracle: the gauge-covariant linear network used as a learned preconditioner
(test infrastructure only).

Not part of the paper: its configurations add a small learned preconditioner
for the main deflated GMRES solves.  Reading used on both sides:

* a "field" is one spinor field (12 complex channels: 4 spin x 3 colour);
* layer l maps f_in fields to f_out fields (1 -> 2 -> 2 -> 1):
      out(x)[f', s', a] = sum_p sum_{f, s} W_p[(f', s'), (f, s)] (T_p in)(x)[f, s, a]
  over the 9 paths p = 0 (identity), +mu (U_mu(x) in(x+mu)) and -mu
  (U_mu(x-mu)^H in(x-mu)), with the antiperiodic sign on hops across the time
  boundary; W_p acts on (field, spin) and as the identity on colour, so the
  network commutes with gauge transformations;
* the network is linear (no activation): a fixed linear operator N, used as a
  right preconditioner inside flexible GMRES, so it can change the cost of a
  solve but never its converged solution;
* loss over pairs (r, e): sum_j ||N(r_j) - e_j||^2 / ||e_j||^2 / npairs.

Parameter vector: for layer 0, 1, 2; for p = 0..8; for o < 4 f_out; for
i < 4 f_in: (Re, Im) of W_p[o][i]  (2304 reals).

Pins (tests/test_oracle_net.py): analytic gradient against central finite
differences; gauge covariance of N; linearity; identity weights give the
identity map.
"""
import numpy as np

from .lattice import neighbour

FIELDS = (1, 2, 2, 1)
NPATH = 9


def layer_shapes():
    return [(NPATH, 4 * FIELDS[l + 1], 4 * FIELDS[l]) for l in range(3)]


def n_params():
    return 2 * sum(np.prod(s) for s in layer_shapes())


def unflatten(theta):
    """Real parameter vector -> list of complex weight arrays W[p][o][i]."""
    out, pos = [], 0
    for shp in layer_shapes():
        cnt = int(np.prod(shp))
        v = np.asarray(theta[pos:pos + 2 * cnt], dtype=np.float64)
        out.append((v[0::2] + 1j * v[1::2]).reshape(shp))
        pos += 2 * cnt
    return out


def flatten(Ws):
    return np.concatenate([np.stack([W.real.ravel(), W.imag.ravel()], axis=1).ravel() for W in Ws])


class Transport:
    """Parallel transports T_p on activations a[..., V, f, 4, 3]."""

    def __init__(self, dims, links, t_antiperiodic=True):
        self.dims = dims
        self.U = np.asarray(links)
        self.fwd, self.bwd, self.sf, self.sb = [], [], [], []
        for mu in range(4):
            f, cf = neighbour(dims, mu, +1)
            b, cb = neighbour(dims, mu, -1)
            self.fwd.append(f)
            self.bwd.append(b)
            self.sf.append(np.where(cf & t_antiperiodic, -1.0, 1.0))
            self.sb.append(np.where(cb & t_antiperiodic, -1.0, 1.0))

    def apply(self, a, p):
        """(T_p a)(x)."""
        if p == 0:
            return a.copy()
        if p <= 4:
            mu = p - 1
            v = a[..., self.fwd[mu], :, :, :]
            return self.sf[mu][:, None, None, None] * np.einsum("xab,...xfsb->...xfsa", self.U[:, mu], v)
        mu = p - 5
        v = a[..., self.bwd[mu], :, :, :]
        Ub = np.conj(np.transpose(self.U[self.bwd[mu], mu], (0, 2, 1)))
        return self.sb[mu][:, None, None, None] * np.einsum("xab,...xfsb->...xfsa", Ub, v)

    def adjoint(self, g, p):
        """T_p^H g (the adjoint with respect to sum conj(u) v)."""
        if p == 0:
            return g.copy()
        out = np.zeros_like(g)
        if p <= 4:
            mu = p - 1
            t = self.sf[mu][:, None, None, None] * np.einsum("xba,...xfsb->...xfsa", np.conj(self.U[:, mu]), g)
            idx = self.fwd[mu]
            out[..., idx, :, :, :] += t
            return out
        mu = p - 5
        Ub = np.conj(np.transpose(self.U[self.bwd[mu], mu], (0, 2, 1)))
        t = self.sb[mu][:, None, None, None] * np.einsum("xba,...xfsb->...xfsa", np.conj(Ub), g)
        out[..., self.bwd[mu], :, :, :] += t
        return out


def to_act(v, V):
    """canonical vectors (..., n) -> activations (..., V, 1, 4, 3)."""
    return np.asarray(v).reshape(v.shape[:-1] + (V, 1, 4, 3))


def from_act(a):
    return a.reshape(a.shape[:-4] + (-1,))


def forward(T, Ws, a, keep=False):
    """Network output; with keep=True also the per-layer transported inputs."""
    cache = []
    for W in Ws:
        Ts = [T.apply(a, p) for p in range(NPATH)]
        if keep:
            cache.append(Ts)
        # out[..., x, f', s', c] = sum_p sum_(f, s) W_p[(f' s'), (f s)] Ts[p][..., x, f, s, c]
        fin = a.shape[-3]
        fout = W.shape[1] // 4
        out = 0
        for p in range(NPATH):
            Wp = W[p].reshape(fout, 4, fin, 4)
            out = out + np.einsum("ostu,...xtuc->...xosc", Wp, Ts[p])
        a = out
    return (a, cache) if keep else a


def loss_and_grad(T, theta, R, E):
    """Loss sum_j ||N(r_j) - e_j||^2/||e_j||^2 / P and its gradient with respect
    to the real parameter vector theta.  R, E: canonical (P, n) complex."""
    Ws = unflatten(theta)
    V = R.shape[-1] // 12
    a0 = to_act(R, V)
    out, cache = forward(T, Ws, a0, keep=True)
    Ea = to_act(E, V)
    P = R.shape[0]
    en = np.sum(np.abs(Ea) ** 2, axis=(-4, -3, -2, -1))          # (P,)
    diff = out - Ea
    loss = float(np.sum(np.sum(np.abs(diff) ** 2, axis=(-4, -3, -2, -1)) / en) / P)
    # g = dL/d(out*) ; for a real loss dL/dRe = 2 Re g, dL/dIm = 2 Im g
    g = diff / (en[:, None, None, None, None] * P)
    grads = []
    for l in (2, 1, 0):
        W = Ws[l]
        Ts = cache[l]
        fout, fin = W.shape[1] // 4, W.shape[2] // 4
        gW = np.zeros_like(W)
        gin = 0
        for p in range(NPATH):
            # out = sum W_p Ts_p  ->  dL/dW_p* = sum g conj(Ts_p) ; dL/dTs_p* = W_p^H g
            gW[p] = np.einsum("Pxosc,Pxtuc->ostu", g, np.conj(Ts[p])).reshape(4 * fout, 4 * fin)
            gTs = np.einsum("ostu,...xosc->...xtuc", np.conj(W[p].reshape(fout, 4, fin, 4)), g)
            gin = gin + T.adjoint(gTs, p)
        grads.append(gW)
        g = gin
    grads = grads[::-1]
    # real gradient: dL/dRe w = 2 Re(dL/dw*), dL/dIm w = 2 Im(dL/dw*)
    return loss, 2.0 * flatten(grads)


def apply_net(T, theta, X):
    """N(x) for canonical (P, n) complex vectors."""
    V = X.shape[-1] // 12
    return from_act(forward(T, unflatten(theta), to_act(X, V)))


def identity_theta():
    """Weights for which the network is the identity map."""
    Ws = []
    for (npath, o, i) in layer_shapes():
        W = np.zeros((npath, o, i), dtype=np.complex128)
        for s in range(4):
            W[0, s, s] = 1.0          # field 0 -> field 0, path 0
        Ws.append(W)
    return flatten(Ws)
