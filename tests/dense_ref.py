"""Independent dense builder of the twisted-mass operator for tiny lattices.

Shares no code with the oracle: the gamma matrices, the hopping term of the
Wilson operator in Eq. (2.1) and the twist are assembled here, as explicit
Kronecker blocks, into a dense (V * nf * 12)^2 matrix indexed like the
canonical layout (site lex = x + Lx*(y + Ly*(z + Lz*t)), then flavour, spin,
colour).  Used to pin the oracle's hop element by element and to supply the
brute-force solves and determinants the even-odd route is checked against.
"""
import numpy as np


def pauli():
    return (np.array([[0, 1], [1, 0]], complex),
            np.array([[0, -1j], [1j, 0]], complex),
            np.array([[1, 0], [0, -1]], complex))


def gammas():
    """Non-relativistic basis of Sec. 2: g_k = [[0, i s_k], [-i s_k, 0]], g_4 = diag(1,1,-1,-1)."""
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, 1j * s], [-1j * s, z]]) for s in pauli()]
    g.append(np.diag([1, 1, -1, -1]).astype(complex))
    return g


def site_index(c, dims):
    x, y, z, t = c
    lx, ly, lz, lt = dims
    return x + lx * (y + ly * (z + lz * t))


def chiral_gammas():
    """A chiral basis (g5 = g1 g2 g3 g4 diagonal), written out:
    g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]], g5 = diag(1, 1, -1, -1)."""
    z = np.zeros((2, 2), complex)
    g = [np.block([[z, -1j * s], [1j * s, z]]) for s in pauli()]
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]).astype(complex))
    return g


def dense_hop(dims, U, nf, tsign=-1.0, dagger=False, gam=None):
    """Dense Wilson hopping matrix D (or D^+) with antiperiodic-t factor tsign
    (gamma matrices of the basis of Sec. 2 unless `gam` gives another set)."""
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    n = nf * 12
    D = np.zeros((V * n, V * n), complex)
    g = gammas() if gam is None else gam
    one = np.eye(4)
    If = np.eye(nf)
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = [x, y, z, t]
                    i = site_index(c, dims)
                    for mu in range(4):
                        cf = list(c); cf[mu] = (c[mu] + 1) % dims[mu]
                        cb = list(c); cb[mu] = (c[mu] - 1) % dims[mu]
                        sf = tsign if (mu == 3 and c[3] == lt - 1) else 1.0
                        sb = tsign if (mu == 3 and c[3] == 0) else 1.0
                        jf, jb = site_index(cf, dims), site_index(cb, dims)
                        Pf = one + g[mu] if dagger else one - g[mu]
                        Pb = one - g[mu] if dagger else one + g[mu]
                        uf = U[mu, t, z, y, x]
                        ub = U[mu, cb[3], cb[2], cb[1], cb[0]].conj().T
                        D[i * n:(i + 1) * n, jf * n:(jf + 1) * n] += sf * np.kron(If, np.kron(Pf, uf))
                        D[i * n:(i + 1) * n, jb * n:(jb + 1) * n] += sb * np.kron(If, np.kron(Pb, ub))
    return D


def twist_block(nf, a, b, sign=1, gam=None):
    """R on (flavour, spin): 1 + i a g5 t3 + b t1, or 1 + i*sign*a*g5 for one flavour."""
    g = gammas() if gam is None else gam
    g5 = g[0] @ g[1] @ g[2] @ g[3]
    if nf == 1:
        return np.eye(4) + 1j * sign * a * g5
    t1, _, t3 = pauli()
    return np.eye(8) + 1j * a * np.kron(t3, g5) + b * np.kron(t1, np.eye(4))


def dense_M(dims, U, kappa, mu, eps=0.0, nf=1, sign=1, tsign=-1.0, gam=None):
    """Dense M = R - kappa D (Eq. 2.1 times 2 kappa) on the canonical index."""
    V = int(np.prod(dims))
    a, b = 2 * kappa * mu, 2 * kappa * eps
    R = np.kron(np.eye(V), np.kron(twist_block(nf, a, b, sign, gam), np.eye(3)))
    return R - kappa * dense_hop(dims, U, nf, tsign, gam=gam)


def parity_index(dims, parity, nf):
    """Indices of the dense vector that belong to sites of the given parity."""
    lx, ly, lz, lt = dims
    idx = []
    n = nf * 12
    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    if (x + y + z + t) % 2 == parity:
                        i = site_index([x, y, z, t], dims)
                        idx.extend(range(i * n, (i + 1) * n))
    return np.array(idx)


def clover_blocks(dims, U, kappa, csw, gam=None):
    """Per-site clover term 1 + i kappa c_sw sum_{mu<nu} sigma_munu F_munu on
    (spin, colour), [V, 12, 12] in lex order, from explicit coordinate loops:
    F = (Q - Q^+)/8, Q the four counter-clockwise plaquette leaves at x."""
    lx, ly, lz, lt = dims
    V = lx * ly * lz * lt
    g = gammas() if gam is None else gam
    out = np.zeros((V, 12, 12), complex)

    def link(mu, c):
        c = [c[i] % dims[i] for i in range(4)]
        return U[mu, c[3], c[2], c[1], c[0]]

    def step(c, mu, d):
        c = list(c)
        c[mu] += d
        return c

    for t in range(lt):
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    c = [x, y, z, t]
                    A = np.eye(12, dtype=complex)
                    for mu in range(4):
                        for nu in range(mu + 1, 4):
                            H = lambda m: m.conj().T
                            cm, cn = step(c, mu, -1), step(c, nu, -1)
                            q = (link(mu, c) @ link(nu, step(c, mu, 1)) @ H(link(mu, step(c, nu, 1))) @ H(link(nu, c))
                                 + link(nu, c) @ H(link(mu, step(cm, nu, 1))) @ H(link(nu, cm)) @ link(mu, cm)
                                 + H(link(mu, cm)) @ H(link(nu, step(cm, nu, -1))) @ link(mu, step(cm, nu, -1)) @ link(nu, cn)
                                 + H(link(nu, cn)) @ link(mu, cn) @ link(nu, step(cn, mu, 1)) @ H(link(mu, c)))
                            F = (q - q.conj().T) / 8
                            sig = 0.5j * (g[mu] @ g[nu] - g[nu] @ g[mu])
                            A = A + 1j * kappa * csw * np.kron(sig, F)
                    out[site_index(c, dims)] = A
    return out


def dense_M_clover(dims, U, kappa, mu, csw, eps=0.0, nf=1, sign=1, tsign=-1.0):
    """Dense twisted-clover M = A + i a g5 t3 + b t1 - kappa D."""
    V = int(np.prod(dims))
    M = dense_M(dims, U, kappa, mu, eps, nf, sign, tsign)
    A = clover_blocks(dims, U, kappa, csw)
    n = 12 * nf
    for i in range(V):
        for f in range(nf):
            o = i * n + 12 * f
            M[o:o + 12, o:o + 12] += A[i] - np.eye(12)
    return M
