"""O1 -- the random diagonal of the Anderson model.

Section 3 (eq. (eigenequation) and the text after it): the diagonal entries
eps_{ijk} are independent draws from the box distribution on [-w/2, w/2].
The paper does not fix a random number generator; the reading used here is
SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), a counter-based generator:

    state_m = seed + m * 0x9E3779B97F4A7C15            (mod 2^64), m = 1, 2, ...
    z = state_m
    z = (z xor (z >> 30)) * 0xBF58476D1CE4E5B9         (mod 2^64)
    z = (z xor (z >> 27)) * 0x94D049BB133111EB         (mod 2^64)
    out_m = z xor (z >> 31)

Site s (0-based, s = i + L*(j + L*k), x fastest) takes the (s+1)-th output:
u_s = (out_{s+1} >> 11) * 2^-53 in [0, 1), eps_s = W * (u_s - 1/2), i.e. the
half-open box [-W/2, W/2) (the closed and half-open boxes differ on a set of
measure zero).
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


def splitmix64_scalar(seed, m):
    """The m-th output (m >= 1) of the stream seeded with ``seed``; Python ints."""
    z = (seed + m * GAMMA) & _MASK
    z = ((z ^ (z >> 30)) * MIX1) & _MASK
    z = ((z ^ (z >> 27)) * MIX2) & _MASK
    return z ^ (z >> 31)


def splitmix64(seed, count, first=1):
    """Outputs number first .. first+count-1 of the stream, as uint64."""
    m = np.arange(first, first + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK) + m * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(MIX1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(MIX2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, count):
    """u_s = top 53 bits of output s+1, scaled by 2^-53 (exact in binary64)."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def disorder(L, W, seed):
    """eps_s = W * (u_s - 1/2) for the L^3 sites, site order x fastest."""
    n = L * L * L
    return W * (uniform01(seed, n) - 0.5)


def hoppings(L, W, seed):
    """Random couplings of the off-diagonal ("inverse") Anderson model (section 8.2,
    Table 6): each bond of the lattice carries its own value, uniform on [-W/2, W/2)
    (the paper: [-1/2, 1/2], W = 1).  The bond from site s to its +x, +y, +z neighbour
    (d = 0, 1, 2) takes output n + 3 s + d + 1 of the same stream as the diagonal, so the
    two never share an output.  Returns t[d, s], shape (3, n)."""
    n = L * L * L
    u = (splitmix64(seed, 3 * n, first=n + 1) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return (W * (u - 0.5)).reshape(n, 3).T.copy()


# the constant diagonal of the off-diagonal model (section 8.2): its transition value
OFFDIAG_DIAGONAL = 1.28


def offdiag_model(L, W, seed):
    """(eps, hop) of the off-diagonal model: constant diagonal 1.28, random bonds."""
    return np.full(L * L * L, OFFDIAG_DIAGONAL), hoppings(L, W, seed)
