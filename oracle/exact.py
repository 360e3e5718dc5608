"""Exact references used to pin the oracle (test infrastructure only).

* exact diagonalisation of a term list in a fixed S^z sector (sparse,
  N <= 18) or in the full space (no symmetry, small N);
* free-fermion closed forms of the open XX chain and the open transverse
  field Ising chain.
"""
import itertools
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from math import comb, pi, cos


def _basis(N, q_target):
    """Bit strings of N spins (bit i = 1 means site i up) with total
    charge q = 2 S^z = q_target; q_target None means the full space."""
    if q_target is None:
        return np.arange(2 ** N, dtype=np.int64)
    assert (N + q_target) % 2 == 0
    n_up = (N + q_target) // 2
    states = []
    for ups in itertools.combinations(range(N), n_up):
        states.append(sum(1 << i for i in ups))
    return np.array(sorted(states), dtype=np.int64)


def _apply(states, amp, site, op):
    bit = (states >> site) & 1
    if op == "I":
        return states, amp
    if op == "Sz":
        return states, amp * np.where(bit == 1, 0.5, -0.5)
    if op == "Sp":
        ok = bit == 0
        return states | (1 << site), amp * ok
    if op == "Sm":
        ok = bit == 1
        return states & ~np.int64(1 << site), amp * ok
    if op == "Sx":
        return states ^ np.int64(1 << site), amp * 0.5
    raise ValueError(op)


def sparse_hamiltonian(terms, N, q_target):
    basis = _basis(N, q_target)
    n = len(basis)
    rows, cols, vals = [], [], []
    for coef, factors in terms:
        st, amp = basis.copy(), np.full(n, coef, dtype=float)
        for site, op in reversed(factors):      # rightmost factor acts first
            st, amp = _apply(st, amp, site, op)
        nz = amp != 0
        if not np.any(nz):
            continue
        pos = np.searchsorted(basis, st[nz])
        assert np.all(basis[pos] == st[nz]), "term leaves the sector"
        rows.append(pos)
        cols.append(np.nonzero(nz)[0])
        vals.append(amp[nz])
    if rows:
        rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    H = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    return H, basis


def ground_state(terms, N, q_target=0, k=1):
    """Lowest eigenpair(s) of H restricted to 2 S^z = q_target."""
    H, basis = sparse_hamiltonian(terms, N, q_target)
    if H.shape[0] <= 400:
        w, v = np.linalg.eigh(H.toarray())
        return w[:k], v[:, :k], basis
    w, v = spla.eigsh(H, k=k, which="SA", tol=1e-14, maxiter=100000)
    o = np.argsort(w)
    return w[o], v[:, o], basis


def xx_chain_energy(N, J=1.0):
    """Open XX chain H = J sum (Sx Sx + Sy Sy): by Jordan-Wigner a hopping
    chain with one-particle energies J cos(k pi/(N+1)); the ground state
    fills all negative levels."""
    return sum(min(0.0, J * cos(k * pi / (N + 1))) for k in range(1, N + 1))


def tfim_chain_energy(N, J=1.0, h=1.0):
    """Open TFIM H = -J sum sz sz - h sum sx (Pauli): E0 = -sum_k s_k(M),
    M the N x N upper bidiagonal matrix with h on the diagonal and J above."""
    M = np.diag(np.full(N, float(h))) + np.diag(np.full(N - 1, float(J)), 1)
    return -float(np.sum(np.linalg.svd(M, compute_uv=False)))


def tfim_chain_dE_dh(N, J=1.0, h=1.0):
    """dE0/dh of the open TFIM from first-order perturbation of the
    singular values: ds_k/dh = u_k . v_k (M depends on h through its diagonal)."""
    M = np.diag(np.full(N, float(h))) + np.diag(np.full(N - 1, float(J)), 1)
    U, s, Vt = np.linalg.svd(M)
    return -float(np.sum(U * Vt.T))


def binomial_count(n_sites, q):
    """Number of spin-1/2 configurations of n_sites with total charge q = 2 S^z."""
    if (n_sites + q) % 2 or abs(q) > n_sites:
        return 0
    return comb(n_sites, (n_sites + q) // 2)
