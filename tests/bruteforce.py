"""Independent numpy formulations used to pin the oracle (test-only).

Nothing here is shared with the oracle or the library: the energy is written
as the Hamiltonian itself with np.roll over the lattice axes, and the
degenerate-temperature dynamics are derived by hand from the Metropolis rule.
"""
import itertools

import numpy as np


def as_cube(v, L):
    """site-major vector (i = x + L(y + Lz)) -> array [z, y, x]"""
    return np.asarray(v).reshape(L, L, L)


def energy(L, J, s):
    """H = -sum over the 3N bonds of J_b s_i s_j (Sec. 2.2, Eq. 1 with h = 0)."""
    S = as_cube(s, L).astype(np.int64)
    Jc = np.asarray(J, dtype=np.int64).reshape(L, L, L, 3)
    E = 0
    for mu, axis in ((0, 2), (1, 1), (2, 0)):   # x is the last array axis
        E -= int(np.sum(Jc[..., mu] * S * np.roll(S, -1, axis=axis)))
    return E


def local_field_unsat(L, J, s):
    """u_i for every site: number of the 6 incident bonds with J s_i s_j = -1."""
    S = as_cube(s, L).astype(np.int64)
    Jc = np.asarray(J, dtype=np.int64).reshape(L, L, L, 3)
    u = np.zeros_like(S)
    for mu, axis in ((0, 2), (1, 1), (2, 0)):
        fwd = Jc[..., mu] * S * np.roll(S, -1, axis=axis)          # bond (i, i+mu)
        bwd = np.roll(Jc[..., mu], 1, axis=axis) * S * np.roll(S, 1, axis=axis)  # bond (i-mu, i)
        u += (fwd < 0).astype(np.int64) + (bwd < 0).astype(np.int64)
    return u.reshape(-1)


def neighbours_plus(L):
    idx = np.arange(L ** 3)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    return np.stack([((x + 1) % L) + L * (y + L * z),
                     x + L * (((y + 1) % L) + L * z),
                     x + L * (y + L * ((z + 1) % L))], axis=1)


def gauge(L, J, spins, tau):
    """s_i -> tau_i s_i, J_(i,i+mu) -> tau_i J tau_(i+mu); tau in +-1 per site."""
    nb = neighbours_plus(L)
    Jg = (np.asarray(J) * tau[:, None] * tau[nb]).astype(np.int8)
    sg = (np.asarray(spins) * tau).astype(np.int8)
    return Jg, sg


def enumerate_energies(L, J):
    """Energy of every one of the 2^N states (small L only)."""
    N = L ** 3
    out = np.empty(2 ** N, dtype=np.int64)
    for n, bits in enumerate(itertools.product((1, -1), repeat=N)):
        out[n] = energy(L, J, np.array(bits[::-1], dtype=np.int64))
    return out


def boltzmann_pdf(energies, beta):
    """Exact P(E) at inverse temperature beta from the enumerated spectrum."""
    vals, counts = np.unique(energies, return_counts=True)
    logw = -beta * vals + np.log(counts)
    logw -= logw.max()
    w = np.exp(logw)
    return vals, w / w.sum()


def colour_classes(L):
    """Proper colour classes as sets of site indices, for the zero-temperature
    dynamics below: parity for even L; for odd L colour (g(x)+g(y)+g(z)) mod 3
    with g(x) = x & 1 except g(L-1) = 2."""
    idx = np.arange(L ** 3)
    x, y, z = idx % L, (idx // L) % L, idx // (L * L)
    if L % 2 == 0:
        col = (x + y + z) & 1
        return [idx[col == c] for c in range(2)]
    g = lambda a: np.where(a == L - 1, 2, a & 1)  # noqa: E731
    col = (g(x) + g(y) + g(z)) % 3
    return [idx[col == c] for c in range(3)]


def zero_temperature_sweeps(L, J, s, n):
    """Metropolis at beta -> infinity: thresholds are 0, so a site flips iff
    dE <= 0, i.e. u >= 3; the colour classes are updated in order."""
    s = np.array(s, dtype=np.int64)
    for _ in range(n):
        for cls in colour_classes(L):
            u = local_field_unsat(L, J, s)
            flip = cls[u[cls] >= 3]
            s[flip] = -s[flip]
    return s.astype(np.int8)


def enumerate_energy_magnetization(L, J):
    """Bond energy and magnetization of every one of the 2^N states (small L only)."""
    N = L ** 3
    E = np.empty(2 ** N, dtype=np.int64)
    M = np.empty(2 ** N, dtype=np.int64)
    for n, bits in enumerate(itertools.product((1, -1), repeat=N)):
        s = np.array(bits[::-1], dtype=np.int64)
        E[n] = energy(L, J, s)
        M[n] = s.sum()
    return E, M


def zero_temperature_sweeps_field(L, J, s, n, h):
    """Metropolis at beta -> infinity in a field h: a site flips iff its cost
    12 - 4u + 2 h s <= 0; the colour classes are updated in order."""
    s = np.array(s, dtype=np.int64)
    for _ in range(n):
        for cls in colour_classes(L):
            u = local_field_unsat(L, J, s)
            cost = 12 - 4 * u[cls] + 2.0 * h * s[cls]
            flip = cls[cost <= 0]
            s[flip] = -s[flip]
    return s.astype(np.int8)
