"""Oracle: the feed-forward network (FFNN) of Sec. 2.2.2 (test infrastructure only).

The paper builds an FFNN from layers that are either affine maps (dense: y = W x + b) or
activations (ln cosh, tanh), and notes that the RBM without visible bias is the single
dense layer with ln cosh activation. Here a network is a sequence of L dense layers, each
followed by its activation:

    z_0 = sigma,   y_l = W_l z_(l-1) + b_l,   z_l = f_l(y_l)   (l = 1 .. L),
    log psi(sigma) = sum_k z_L,k

(the last layer's outputs summed; with L = 1 and f = ln cosh this is the RBM without
visible bias, including its dropped constant). Parameters are complex (or real) and packed
layer by layer as [b_l (n_l) | W_l (n_l x n_(l-1), row j, column k)].

Log-derivatives by the chain rule (backpropagation), with g_l = d log psi / d y_l:
g_L = f_L'(y_L), g_l = f_l'(y_l) * (W_(l+1)^T g_(l+1)); then O_(b_l) = g_l and
O_(W_l),jk = g_l,j z_(l-1),k. The derivative of ln cosh is tanh, that of tanh is 1 - tanh^2.

Pins (tests/test_oracle_ffnn.py): one ln cosh layer equals the RBM with zero visible bias
(log psi and every log-derivative); a first tanh layer with tiny weights equals, within its
O(eps^3) bound, the RBM whose weights are the product of the two layers; log-derivatives
against central finite differences for two- and three-layer networks; with zero biases and
ln cosh last, log psi is even under sigma -> -sigma; local energies of the network against
the dense Hamiltonian (sum_s p(s) E_loc(s) = <psi|H|psi> / <psi|psi>).
"""
import numpy as np

from . import rbm

LNCOSH = 0
TANH = 1


def act(code, y):
    return rbm.ln_cosh(y) if code == LNCOSH else np.tanh(y)


def act_deriv(code, y):
    t = np.tanh(y)
    return t if code == LNCOSH else 1.0 - t * t


class FFNN:
    """A network over n_sites spins with layer widths sizes[0..L-1] and activations."""

    def __init__(self, n_sites, sizes, acts):
        if len(sizes) != len(acts) or not sizes:
            raise ValueError("one activation per layer, at least one layer")
        self.n_sites = int(n_sites)
        self.sizes = [int(s) for s in sizes]
        self.acts = [int(a) for a in acts]

    @property
    def widths(self):
        return [self.n_sites] + self.sizes

    @property
    def n_params(self):
        w = self.widths
        return sum(w[l + 1] * (1 + w[l]) for l in range(len(self.sizes)))

    def unpack(self, params):
        p = np.asarray(params)
        if p.shape != (self.n_params,):
            raise ValueError("params has %s entries, expected %d" % (p.shape, self.n_params))
        out, off, w = [], 0, self.widths
        for l in range(len(self.sizes)):
            m, k = w[l + 1], w[l]
            b = p[off:off + m]
            W = p[off + m:off + m + m * k].reshape(m, k)
            out.append((b, W))
            off += m * (1 + k)
        return out

    def pack(self, layers):
        return np.concatenate([np.concatenate([b, W.reshape(-1)]) for b, W in layers])

    def forward(self, params, sigma):
        """Pre-activations ys[l] and layer inputs zs[l] (zs[0] = sigma), each [n, width]."""
        z = np.asarray(sigma, dtype=np.float64)
        ys, zs = [], [z]
        for (b, W), a in zip(self.unpack(params), self.acts):
            y = z @ W.T + b[None, :]
            z = act(a, y)
            ys.append(y)
            zs.append(z)
        return ys, zs

    def log_psi(self, params, sigma):
        _, zs = self.forward(params, sigma)
        return zs[-1].sum(axis=1)

    def log_derivatives(self, params, sigma):
        """O[s, k] = d log psi(sigma_s) / d p_k: [n, P] by backpropagation."""
        layers = self.unpack(params)
        ys, zs = self.forward(params, sigma)
        L = len(layers)
        gs = [None] * L
        gs[L - 1] = act_deriv(self.acts[L - 1], ys[L - 1])
        for l in range(L - 2, -1, -1):
            W_next = layers[l + 1][1]
            gs[l] = act_deriv(self.acts[l], ys[l]) * (gs[l + 1] @ W_next)
        n = gs[0].shape[0]
        cols = []
        for l in range(L):
            cols.append(gs[l])
            cols.append((gs[l][:, :, None] * zs[l][:, None, :]).reshape(n, -1))
        return np.concatenate(cols, axis=1)

    def jvp(self, params, sigma, v):
        return self.log_derivatives(params, sigma) @ np.asarray(v)

    def vjp(self, params, sigma, u):
        return np.conj(self.log_derivatives(params, sigma)).T @ np.asarray(u)


class RBMMachine:
    """The plain RBM behind the same interface (log_psi, log_derivatives)."""

    def __init__(self, n_sites, n_hidden):
        self.n_sites, self.n_hidden = n_sites, n_hidden

    def log_psi(self, params, sigma):
        return rbm.log_psi(params, sigma, self.n_sites, self.n_hidden)

    def log_derivatives(self, params, sigma):
        return rbm.log_derivatives(params, sigma, self.n_sites, self.n_hidden)
