"""Lattices and Hamiltonian term lists (oracle; test infrastructure only).

Spin-1/2 local basis, ordered by ascending charge q = 2 S^z:
index 0 = down (q = -1), index 1 = up (q = +1).

A Hamiltonian is a list of terms ``(coef, ((site, op), ...))`` with the
sites strictly increasing; each term is ``coef * prod op_site``.

Geometry (paper Sec. III, cylinders periodic in y and open in x):
sites are numbered column by column in a snake, site(x, y) = x*Ly + y for
even x and x*Ly + (Ly-1-y) for odd x.
"""
import numpy as np

SPIN_HALF_Q = (-1, 1)

OPS = {
    "I": np.eye(2),
    "Sz": np.diag([-0.5, 0.5]),
    "Sp": np.array([[0.0, 0.0], [1.0, 0.0]]),   # |up><down|
    "Sm": np.array([[0.0, 1.0], [0.0, 0.0]]),   # |down><up|
    "Sx": np.array([[0.0, 0.5], [0.5, 0.0]]),
}


# Spin 1 (the Fig. 3 chains): local states m = -1, 0, 1, charges q = 2 m.
SPIN_ONE_Q = (-2, 0, 2)
_R2 = np.sqrt(2.0)
OPS_S1 = {
    "I": np.eye(3),
    "Sz": np.diag([-1.0, 0.0, 1.0]),
    "Sp": np.array([[0.0, 0.0, 0.0], [_R2, 0.0, 0.0], [0.0, _R2, 0.0]]),   # S+|m> = sqrt(2)|m+1>
    "Sm": np.array([[0.0, _R2, 0.0], [0.0, 0.0, _R2], [0.0, 0.0, 0.0]]),
}


def snake_site(x, y, Ly):
    return x * Ly + (y if x % 2 == 0 else Ly - 1 - y)


def chain_bonds(N):
    return [(i, i + 1) for i in range(N - 1)]


def square_cylinder_bonds(Lx, Ly):
    """Nearest-neighbour bonds of an Lx x Ly cylinder (open x, periodic y)."""
    bonds = set()
    for x in range(Lx):
        for y in range(Ly):
            if Ly > 2 or (Ly == 2 and y == 0):
                bonds.add(tuple(sorted((snake_site(x, y, Ly), snake_site(x, (y + 1) % Ly, Ly)))))
            if x + 1 < Lx:
                bonds.add(tuple(sorted((snake_site(x, y, Ly), snake_site(x + 1, y, Ly)))))
    return sorted(bonds)


def triangular_cylinder_bonds(Lx, Ly):
    """Triangular lattice on an Lx x Ly cylinder: the square bonds plus the
    diagonal (x, y)-(x+1, y-1 mod Ly)."""
    bonds = set(square_cylinder_bonds(Lx, Ly))
    if Ly >= 2:
        for x in range(Lx - 1):
            for y in range(Ly):
                bonds.add(tuple(sorted((snake_site(x, y, Ly), snake_site(x + 1, (y - 1) % Ly, Ly)))))
    return sorted(bonds)


def square_plaquette_bond_pairs(Lx, Ly):
    """Pairs of bonds on opposite sides of every elementary square plaquette
    of the cylinder (the sum in the pure Q2 model, Eq. eqn:q2)."""
    assert Ly >= 3, "plaquettes need Ly >= 3 on a cylinder"
    pairs = []
    for x in range(Lx - 1):
        for y in range(Ly):
            y1 = (y + 1) % Ly
            p00, p10 = snake_site(x, y, Ly), snake_site(x + 1, y, Ly)
            p01, p11 = snake_site(x, y1, Ly), snake_site(x + 1, y1, Ly)
            pairs.append(((p00, p10), (p01, p11)))   # two horizontal bonds
            pairs.append(((p00, p01), (p10, p11)))   # two vertical bonds
    return pairs


def _dot_parts(i, j):
    """S_i . S_j = Sz Sz + (Sp Sm + Sm Sp)/2 as (coef, ops_i, ops_j)."""
    return [(1.0, "Sz", "Sz"), (0.5, "Sp", "Sm"), (0.5, "Sm", "Sp")]


def _sorted_term(coef, factors):
    factors = sorted(factors)
    sites = [s for s, _ in factors]
    assert len(set(sites)) == len(sites), "repeated site in a term"
    return (coef, tuple(factors))


def xxz_terms(bonds, J=1.0, Delta=1.0):
    """H = J sum_<ij> (Sx Sx + Sy Sy + Delta Sz Sz).  The S^z S^z term is kept
    even at Delta = 0 so that the MPO structure does not depend on couplings."""
    terms = []
    for i, j in bonds:
        i, j = min(i, j), max(i, j)
        terms.append((J * Delta, ((i, "Sz"), (j, "Sz"))))
        terms.append((0.5 * J, ((i, "Sp"), (j, "Sm"))))
        terms.append((0.5 * J, ((i, "Sm"), (j, "Sp"))))
    return terms


def heisenberg_terms(bonds, J=1.0):
    return xxz_terms(bonds, J, 1.0)


def tfim_terms(N, J=1.0, h=1.0):
    """Open transverse-field Ising chain H = -J sum sz sz - h sum sx with
    Pauli matrices (sz = 2 Sz, sx = 2 Sx).  Does not conserve S^z."""
    terms = [(-4.0 * J, ((i, "Sz"), (i + 1, "Sz"))) for i in range(N - 1)]
    terms += [(-2.0 * h, ((i, "Sx"),)) for i in range(N)]
    return terms


def tri_sublattice(x, y):
    """Three-colouring of the triangular cylinder (bonds (x,y)-(x,y+1),
    (x,y)-(x+1,y), (x,y)-(x+1,y-1)): neighbours differ by 1 or 2 mod 3."""
    return (x - y) % 3


def triangular_pin_terms(Lx, Ly, h):
    """Sec. III pinning of the triangular study: the field -h S^z on the sites
    of the open edge columns that belong to sublattice 0 (the paper: h = J/2)."""
    assert Ly % 3 == 0
    return [(-h, ((snake_site(x, y, Ly), "Sz"),)) for x in (0, Lx - 1) for y in range(Ly)
            if tri_sublattice(x, y) == 0]


def jq2_pin_terms(Lx, Ly, Q=1.0, pin=1.0):
    """Sec. III strong pinning of the J-Q2 study: pin * (Q/4)(S_r.S_{r+y} - 1/4)
    on every vertical bond of the two open edge columns; the constant is
    returned separately."""
    terms, const = [], 0.0
    for x in (0, Lx - 1):
        for y in range(Ly):
            a, b = snake_site(x, y, Ly), snake_site(x, (y + 1) % Ly, Ly)
            for c, oa, ob in _dot_parts(a, b):
                terms.append(_sorted_term(pin * 0.25 * Q * c, [(a, oa), (b, ob)]))
            const += -pin * Q / 16.0
    return terms, const


def jq2_terms(Lx, Ly, J=1.0, Q=1.0, pin=0.0):
    """J-Q2 model on the square cylinder:
    H = J sum_<ij> S_i.S_j - Q sum_plaq (S_a.S_b - 1/4)(S_c.S_d - 1/4),
    the Q sum running over both pairs of opposite plaquette bonds
    (pure-Q2 form of Eq. eqn:q2 plus the Heisenberg J term), plus the edge
    pinning of Sec. III when pin != 0."""
    terms = heisenberg_terms(square_cylinder_bonds(Lx, Ly), J)
    const = 0.0
    for (a, b), (c, d) in square_plaquette_bond_pairs(Lx, Ly):
        # (S_a.S_b)(S_c.S_d)
        for ca, oa, ob in _dot_parts(a, b):
            for cc, oc, od in _dot_parts(c, d):
                terms.append(_sorted_term(-Q * ca * cc, [(a, oa), (b, ob), (c, oc), (d, od)]))
        # -1/4 (S_a.S_b + S_c.S_d)
        for (x, y) in ((a, b), (c, d)):
            for cx, ox, oy in _dot_parts(x, y):
                terms.append(_sorted_term(Q * 0.25 * cx, [(x, ox), (y, oy)]))
        const += -Q / 16.0
    if pin:
        pt, pc = jq2_pin_terms(Lx, Ly, Q, pin)
        terms += pt
        const += pc
    terms.append((const, ((0, "I"),)))      # kept at Q = 0: structure independent of couplings
    return terms
