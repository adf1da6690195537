"""Independent dense constructions used to pin the oracle (tiny lattices only).

Nothing here calls the oracle.  The Wilson-Dirac matrix is assembled from the
covariant difference operators of Appendix A (eq. wdo and the definitions of
nabla_mu, nabla*_mu that follow it) as products of matrices, not from the
per-site hopping formula the oracle uses, and the gamma matrices are rebuilt
here from the Pauli matrices.
"""
import numpy as np


def pauli():
    return [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]], complex),
            np.array([[1, 0], [0, -1]], complex)]


def gammas():
    """Chiral basis: gamma_0 = [[0,-1],[-1,0]], gamma_k = [[0,-i s_k],[i s_k,0]]."""
    Z = np.zeros((2, 2), complex)
    I2 = np.eye(2)
    g = [np.block([[Z, -I2], [-I2, Z]])]
    for s in pauli():
        g.append(np.block([[Z, -1j * s], [1j * s, Z]]))
    return g


def _idx(L, x):
    return ((x[0] * L[1] + x[1]) * L[2] + x[2]) * L[3] + x[3]


def nabla(U, L, mu, antiperiodic=True):
    """Forward covariant difference nabla_mu on site-colour space (3V x 3V)."""
    V = int(np.prod(L))
    N = np.zeros((V, 3, V, 3), complex)
    for s, x in enumerate(np.ndindex(*L)):
        y = list(x)
        y[mu] += 1
        sign = 1.0
        if y[mu] == L[mu]:
            y[mu] = 0
            if mu == 0 and antiperiodic:
                sign = -1.0
        N[s, :, _idx(L, y), :] += sign * U[s, mu]
        N[s, :, s, :] -= np.eye(3)
    return N.reshape(3 * V, 3 * V)


def nabla_star(U, L, mu, antiperiodic=True):
    """Backward covariant difference nabla*_mu on site-colour space."""
    V = int(np.prod(L))
    N = np.zeros((V, 3, V, 3), complex)
    for s, x in enumerate(np.ndindex(*L)):
        y = list(x)
        y[mu] -= 1
        sign = 1.0
        if y[mu] < 0:
            y[mu] = L[mu] - 1
            if mu == 0 and antiperiodic:
                sign = -1.0
        sy = _idx(L, y)
        N[s, :, s, :] += np.eye(3)
        N[s, :, sy, :] -= sign * U[sy, mu].conj().T
    return N.reshape(3 * V, 3 * V)


def spin_kron(Gm, N, V):
    """Full operator on index (site, spin, colour) from a 4x4 spin matrix and a site-colour operator."""
    N4 = N.reshape(V, 3, V, 3)
    return np.einsum("ab,sitj->saitbj", Gm, N4).reshape(12 * V, 12 * V)


def wilson_dirac(U, L, kappa, antiperiodic=True):
    """D = D_w + m0, D_w = 1/2 sum_mu {gamma_mu (nabla*_mu + nabla_mu) - nabla*_mu nabla_mu}."""
    V = int(np.prod(L))
    g = gammas()
    m0 = 1.0 / (2.0 * kappa) - 4.0
    D = m0 * np.eye(12 * V, dtype=complex)
    for mu in range(4):
        Nf = nabla(U, L, mu, antiperiodic)
        Nb = nabla_star(U, L, mu, antiperiodic)
        D += 0.5 * spin_kron(g[mu], Nb + Nf, V)
        D -= 0.5 * spin_kron(np.eye(4), Nb @ Nf, V)
    return D


def domain_indices(L, lo, hi):
    """Indices (into the 12V vector) of the spin-colour components of sites in [lo,hi)."""
    out = []
    for s, x in enumerate(np.ndindex(*L)):
        if all(lo[m] <= x[m] < hi[m] for m in range(4)):
            out.extend(range(12 * s, 12 * s + 12))
    return np.array(out, dtype=np.int64)
