"""Plain FP64 DMRG on U(1) block-sparse tensors (oracle; test infrastructure only).

Follows the paper's Sec. II step by step:
  * environments ("projected operators") transformed while sweeping;
  * two-site wavefunction Psi^{a2 s3 s4 a4} (Eq. eqn:wf) optimised by a few
    Davidson steps with the Hamiltonian projected into |a2>|s3>|s4>|a4>;
  * SVD Psi = A Lambda B (Eq. eqn:svd), keep the m largest singular values,
    computed with the accurate recursive SVD of the Appendix;
  * at a shared bond Psi = (A Lambda) V (Lambda B), V = Lambda^{-1}
    (Eqs. eqn:inverse, eqn:isvd); merge Psi' = psi'_L V psi'_R with the
    original V (Eq. eqn:merge);
  * n real-space regions swept in the staggered pattern of Fig. 4.

Every contraction is written block by block with plain matrix products; no
fusion or reordering beyond associating a chain of products.
"""
from dataclasses import dataclass, field
import numpy as np
import scipy.linalg as sla

from .blocks import (Bond, site_keys, two_site_keys, env_keys, site_shape,
                     two_site_shape, flatten, unflatten, norm)


# ----------------------------------------------------------------------------
# environments
# ----------------------------------------------------------------------------

def left_boundary():
    return {(0, 0): np.ones((1, 1))}


def right_boundary(q_target):
    return {(q_target, 0): np.ones((1, 1))}


def update_L(L, A, W, phys_q, dl, dr):
    """L'[b, w', b'] = sum A[a, s, b] L[a, w, a'] W[w, s, s', w'] A[a', s', b']
    (real tensors, so the bra copy of A is A itself).  dl, dr: channel
    charges of the MPO bonds left and right of the site."""
    d = len(phys_q)
    out = {}
    for (qa, w), Lb in L.items():
        qk = qa - dl[w]
        for s in range(d):
            Ab = A.get((qa, s))
            if Ab is None:
                continue
            qb = qa + phys_q[s]
            for t in range(d):
                Ak = A.get((qk, t))
                if Ak is None:
                    continue
                coefs = W[w, s, t, :]
                nz = np.nonzero(coefs)[0]
                if len(nz) == 0:
                    continue
                X = Ab.T @ Lb @ Ak
                qbk = qk + phys_q[t]
                for w2 in nz:
                    assert qb - qbk == dr[w2], "MPO entry violates charge conservation"
                    key = (qb, int(w2))
                    out[key] = out.get(key, 0.0) + coefs[w2] * X
    return out


def update_R(R, B, W, phys_q, dl, dr):
    """R'[a, w, a'] = sum B[a, s, b] W[w, s, s', w'] R[b, w', b'] B[a', s', b']."""
    d = len(phys_q)
    out = {}
    for (qb, w2), Rb in R.items():
        qbk = qb - dr[w2]
        for s in range(d):
            qa = qb - phys_q[s]
            Bb = B.get((qa, s))
            if Bb is None:
                continue
            for t in range(d):
                qak = qbk - phys_q[t]
                Bk = B.get((qak, t))
                if Bk is None:
                    continue
                coefs = W[:, s, t, w2]
                nz = np.nonzero(coefs)[0]
                if len(nz) == 0:
                    continue
                X = Bb @ Rb @ Bk.T
                for w in nz:
                    assert qa - qak == dl[w], "MPO entry violates charge conservation"
                    key = (qa, int(w))
                    out[key] = out.get(key, 0.0) + coefs[w] * X
    return out


# ----------------------------------------------------------------------------
# two-site effective Hamiltonian
# ----------------------------------------------------------------------------

def two_site_mpo(W1, W2):
    """W12[w, s1, t1, s2, t2, w2] = sum_c W1[w, s1, t1, c] W2[c, s2, t2, w2]."""
    return np.einsum("astc,cuvb->astuvb", W1, W2)


def heff_apply(L, R, W1, W2, psi, bl, br, phys_q, dl, dr):
    """y = H_eff psi for the two-site wavefunction on bonds (bl, br):
    y[a, s1, s2, b] = sum L[a, w, a'] W1[w, s1, t1, c] W2[c, s2, t2, w2]
                          R[b, w2, b'] psi[a', t1, t2, b'].
    Returned with every allowed block present."""
    d = len(phys_q)
    W12 = two_site_mpo(W1, W2)
    keys = two_site_keys(bl, br, phys_q)
    y = {k: np.zeros(two_site_shape(k, bl, br, phys_q)) for k in keys}
    for (qa, w), Lb in L.items():
        qk = qa - dl[w]
        for t1 in range(d):
            for t2 in range(d):
                pb = psi.get((qk, t1, t2))
                if pb is None:
                    continue
                T = None
                for s1 in range(d):
                    for s2 in range(d):
                        out = y.get((qa, s1, s2))
                        if out is None:
                            continue
                        coefs = W12[w, s1, t1, s2, t2, :]
                        nz = np.nonzero(coefs)[0]
                        if len(nz) == 0:
                            continue
                        if T is None:
                            T = Lb @ pb
                        qb = qa + phys_q[s1] + phys_q[s2]
                        for w2 in nz:
                            Rb = R.get((qb, int(w2)))
                            if Rb is None:
                                continue
                            assert qb - dr[w2] == qk + phys_q[t1] + phys_q[t2]
                            out += coefs[w2] * (T @ Rb.T)
    return y


def heff_apply_rows(L, R, W1, W2, psi, bl, br, phys_q, dl, dr, key, rows):
    """Selected rows of one output block of heff_apply: y[key][rows, :].
    Row a of y depends on row a of L[(q_a, w)] only, so the same sum is taken
    with those rows alone (for checking full-size products one row at a
    time)."""
    d = len(phys_q)
    W12 = two_site_mpo(W1, W2)
    qa, s1, s2 = key
    rows = np.asarray(rows)
    out = np.zeros((len(rows),) + two_site_shape(key, bl, br, phys_q)[1:])
    qb = qa + phys_q[s1] + phys_q[s2]
    for w in range(W12.shape[0]):
        Lb = L.get((qa, w))
        if Lb is None:
            continue
        qk = qa - dl[w]
        for t1 in range(d):
            for t2 in range(d):
                pb = psi.get((qk, t1, t2))
                if pb is None:
                    continue
                coefs = W12[w, s1, t1, s2, t2, :]
                nz = np.nonzero(coefs)[0]
                if len(nz) == 0:
                    continue
                T = Lb[rows] @ pb
                for w2 in nz:
                    Rb = R.get((qb, int(w2)))
                    if Rb is None:
                        continue
                    assert qb - dr[w2] == qk + phys_q[t1] + phys_q[t2]
                    out += coefs[w2] * (T @ Rb.T)
    return out


def heff_diag(L, R, W1, W2, bl, br, phys_q, dl, dr):
    """Diagonal of H_eff (Davidson preconditioner)."""
    d = len(phys_q)
    W12 = two_site_mpo(W1, W2)
    keys = two_site_keys(bl, br, phys_q)
    out = {}
    for k in keys:
        qa, s1, s2 = k
        qb = qa + phys_q[s1] + phys_q[s2]
        acc = np.zeros(two_site_shape(k, bl, br, phys_q))
        for w in range(W12.shape[0]):
            if dl[w] != 0 or (qa, w) not in L:
                continue
            la = np.diag(L[(qa, w)])
            for w2 in range(W12.shape[5]):
                c = W12[w, s1, s1, s2, s2, w2]
                if c == 0 or dr[w2] != 0 or (qb, w2) not in R:
                    continue
                acc += c * np.outer(la, np.diag(R[(qb, w2)]))
        out[k] = acc
    return out


def heff_dense(L, R, W1, W2, bl, br, phys_q, dl, dr):
    """Explicit H_eff matrix over the flattened two-site basis (tiny shapes
    only): built from dense L, W1 W2, R with one einsum, independently of the
    block loops of heff_apply."""
    d = len(phys_q)
    ml, mr = bl.total(), br.total()
    Ld = np.zeros((ml, len(dl), ml))
    for (q, w), blk in L.items():
        o1, o2 = bl.offset(q), bl.offset(q - dl[w])
        Ld[o1:o1 + blk.shape[0], w, o2:o2 + blk.shape[1]] = blk
    Rd = np.zeros((mr, len(dr), mr))
    for (q, w), blk in R.items():
        o1, o2 = br.offset(q), br.offset(q - dr[w])
        Rd[o1:o1 + blk.shape[0], w, o2:o2 + blk.shape[1]] = blk
    W12 = two_site_mpo(W1, W2)
    H = np.einsum("awx,wsturz,bzy->asubxtry", Ld, W12, Rd)
    H = H.reshape(ml * d * d * mr, ml * d * d * mr)
    # restrict to the allowed entries, in the canonical flattened order
    keys = two_site_keys(bl, br, phys_q)
    idx = []
    for (qa, s1, s2) in keys:
        qb = qa + phys_q[s1] + phys_q[s2]
        oa, ob = bl.offset(qa), br.offset(qb)
        for a in range(bl.dim(qa)):
            for b in range(br.dim(qb)):
                idx.append((((oa + a) * d + s1) * d + s2) * mr + ob + b)
    idx = np.array(idx, dtype=np.int64)
    return H[np.ix_(idx, idx)], H, idx


# ----------------------------------------------------------------------------
# eigensolvers
# ----------------------------------------------------------------------------

@dataclass
class DavidsonParams:
    max_matvec: int = 20
    tol: float = 1e-10         # on the residual norm ||H x - theta x||
    max_sub: int = 8           # restart to the Ritz vector at this size


def davidson(matvec, x0, diag, p):
    """Lowest eigenpair of a symmetric operator (Davidson 1975):
    Rayleigh-Ritz on an orthonormal basis V, residual r = H x - theta x,
    diagonal-preconditioned correction t = r / (diag - theta) orthogonalised
    against V twice (classical Gram-Schmidt), restart to the current Ritz
    vector when the basis reaches max_sub vectors.  The Ritz vector's sign is
    chosen so that its overlap with the starting vector is >= 0."""
    x = x0 / np.linalg.norm(x0)
    V = [x]
    HV = [matvec(x)]
    nmv = 1
    while True:
        k = len(V)
        Vm, HVm = np.array(V), np.array(HV)
        G = Vm @ HVm.T
        G = 0.5 * (G + G.T)
        w, C = np.linalg.eigh(G)
        theta, c = w[0], C[:, 0]
        if c[0] < 0:
            c = -c
        x = c @ Vm
        hx = c @ HVm
        r = hx - theta * x
        rn = float(np.linalg.norm(r))
        if rn <= p.tol or nmv >= p.max_matvec:
            break
        den = diag - theta
        den = np.where(np.abs(den) < 1e-8, np.copysign(1e-8, den), den)
        t = r / den
        for _ in range(2):
            t = t - Vm.T @ (Vm @ t)
        tn = np.linalg.norm(t)
        if tn < 1e-14:
            break
        t = t / tn
        if k >= p.max_sub:
            xn = np.linalg.norm(x)
            V, HV = [x / xn], [hx / xn]
        V.append(t)
        HV.append(matvec(t))
        nmv += 1
    return float(theta), x / np.linalg.norm(x), rn, nmv


def lanczos_lowest(matvec, x0, n_iter=60, tol=1e-13):
    """Plain Lanczos with full reorthogonalisation; lowest Ritz value of the
    tridiagonal matrix.  Independent second eigensolver for the pins."""
    q = x0 / np.linalg.norm(x0)
    Q, alphas, betas = [q], [], []
    for j in range(n_iter):
        w = matvec(Q[-1])
        a = float(Q[-1] @ w)
        alphas.append(a)
        w = w - a * Q[-1] - (betas[-1] * Q[-2] if betas else 0.0)
        Qm = np.array(Q)
        w = w - Qm.T @ (Qm @ w)
        b = float(np.linalg.norm(w))
        if b < tol or len(Q) == len(x0):
            break
        betas.append(b)
        Q.append(w / b)
    T = np.diag(alphas) + np.diag(betas[:len(alphas) - 1], 1) + np.diag(betas[:len(alphas) - 1], -1)
    return float(np.linalg.eigvalsh(T)[0])


# ----------------------------------------------------------------------------
# accurate SVD (Appendix) and truncation
# ----------------------------------------------------------------------------

def svd_gesvd(M):
    """Standard backward-stable SVD (LAPACK dgesvd)."""
    U, s, Vt = sla.svd(M, full_matrices=False, lapack_driver="gesvd")
    return U, s, Vt


def svd_rho(M):
    """SVD via the eigendecomposition of rho = M M^T = A Lambda^2 A^T; B from
    the rows of A^T M, normalised and orthogonalised (Appendix step 1,
    second option).  Small singular values are inaccurate in relative terms."""
    n, m = M.shape
    k = min(n, m)
    ev, A = np.linalg.eigh(M @ M.T)
    order = np.argsort(ev)[::-1][:k]
    ev, A = ev[order], A[:, order]
    lam = np.sqrt(np.clip(ev, 0.0, None))
    Y = A.T @ M
    B = np.zeros_like(Y)
    for i in range(k):
        v = Y[i].copy()
        for _ in range(2):
            v = v - B[:i].T @ (B[:i] @ v)
        nv = np.linalg.norm(v)
        if nv > 0:
            B[i] = v / nv
        else:                               # no information left: any unit vector orthogonal to the others
            e = np.zeros(m)
            for j in range(m):
                e[:] = 0.0
                e[j] = 1.0
                for _ in range(2):
                    e = e - B[:i].T @ (B[:i] @ e)
                if np.linalg.norm(e) > 0.5:
                    break
            B[i] = e / np.linalg.norm(e)
    return A, lam, B


def accurate_svd(M, eps=1e-4, step1=svd_gesvd, depth=0):
    """Appendix algorithm.  (1) SVD M = A Lambda B by a standard method.
    (2) find the first p with lambda_p / lambda_1 < eps (0-based).  (3) if none,
    done.  (4) X = A^T M B^T restricted to the trailing indices p.. .
    (5) recurse on X -> (A~, L~, B~).  (6) A[:, p:] <- A[:, p:] A~,
    B[p:] <- B~ B[p:], lambda[p:] <- L~.  Singular values are returned sorted
    in descending order (with A, B permuted alike)."""
    A, lam, B = step1(M)
    if lam.size == 0 or lam[0] == 0.0:
        return A, lam, B
    small = np.nonzero(lam < eps * lam[0])[0]
    if small.size == 0:
        return A, lam, B
    p = int(small[0])
    X = A[:, p:].T @ M @ B[p:, :].T
    At, lt, Bt = accurate_svd(X, eps, step1, depth + 1)
    A = A.copy()
    B = B.copy()
    lam = lam.copy()
    A[:, p:] = A[:, p:] @ At
    B[p:, :] = Bt @ B[p:, :]
    lam[p:] = lt
    order = np.argsort(-lam, kind="stable")
    return A[:, order], lam[order], B[order]


@dataclass
class TruncResult:
    bond: Bond
    A: dict
    B: dict
    lam: dict             # q -> kept singular values (renormalised)
    center: dict = None   # AΛ (mode left) or ΛB (mode right)
    left: dict = None     # AΛ (mode split)
    right: dict = None    # ΛB (mode split)
    V: dict = None        # q -> 1/lambda (mode split)
    discarded: float = 0.0
    n_floored: int = 0


def svd_truncate(psi, bl, br, phys_q, max_m, mode, cutoff=1e-12, eps=1e-4,
                 v_floor=1e-12, step1=svd_gesvd):
    """Truncated SVD of the two-site wavefunction viewed as the (m d) x (d m)
    matrix Psi^{(a s1),(s2 b)} (Eq. eqn:svd), block-diagonal in the middle
    charge q = q_a + q_s1.  Rows of a sector run over s1 ascending then a,
    columns over s2 ascending then b.

    Truncation: keep the max_m largest singular values over all sectors,
    dropping lambda < cutoff * lambda_max; ties broken by (lambda descending,
    charge ascending, in-sector index ascending).  The kept Lambda is
    renormalised to sum lambda^2 = 1.
    mode 'right': A kept, centre Lambda B moves right;
    mode 'left' : B kept, centre A Lambda moves left;
    mode 'split': both A Lambda and Lambda B plus V = 1/lambda, floored at
                  1/(v_floor * lambda_max) (Eqs. eqn:inverse, eqn:isvd)."""
    d = len(phys_q)
    mids = sorted({qa + phys_q[s1] for (qa, s1, s2) in psi.keys()})
    dec = {}
    for qm in mids:
        rows = [(s1, qm - phys_q[s1]) for s1 in range(d) if bl.has(qm - phys_q[s1])]
        cols = [(s2, qm + phys_q[s2]) for s2 in range(d) if br.has(qm + phys_q[s2])]
        if not rows or not cols:
            continue
        M = np.block([[psi.get((qa, s1, s2), np.zeros((bl.dim(qa), br.dim(qb))))
                       for (s2, qb) in cols] for (s1, qa) in rows])
        U, lam, Vt = accurate_svd(M, eps, step1)
        dec[qm] = (rows, cols, U, lam, Vt)
    cand = [(-lam[i], qm, i) for qm, (_, _, _, lam, _) in dec.items() for i in range(len(lam))]
    cand.sort()
    total = sum(l * l for (l, _, _) in cand)
    lmax = -cand[0][0] if cand else 0.0
    kept = {}
    for (nl, qm, i) in cand[:max_m]:
        if -nl >= cutoff * lmax and -nl > 0.0:
            kept[qm] = kept.get(qm, 0) + 1
    kept_w = sum(float(np.sum(dec[qm][3][:k] ** 2)) for qm, k in kept.items())
    scale = 1.0 / np.sqrt(kept_w)
    bond = Bond(kept)
    A, B, lamd = {}, {}, {}
    for qm, k in kept.items():
        rows, cols, U, lam, Vt = dec[qm]
        lamd[qm] = lam[:k] * scale
        r0 = 0
        for (s1, qa) in rows:
            A[(qa, s1)] = U[r0:r0 + bl.dim(qa), :k].copy()
            r0 += bl.dim(qa)
        c0 = 0
        for (s2, qb) in cols:
            B[(qm, s2)] = Vt[:k, c0:c0 + br.dim(qb)].copy()
            c0 += br.dim(qb)
    res = TruncResult(bond=bond, A=A, B=B, lam=lamd, discarded=max(0.0, 1.0 - kept_w / total))
    lB = {k: lamd[k[0]][:, None] * v for k, v in B.items()}
    Al = {k: v * lamd[k[0] + phys_q[k[1]]][None, :] for k, v in A.items()}
    if mode == "right":
        res.center = lB
    elif mode == "left":
        res.center = Al
    elif mode == "split":
        res.left, res.right = Al, lB
        lm = max(float(np.max(v)) for v in lamd.values())
        res.V = {}
        for q, v in lamd.items():
            fl = np.maximum(v, v_floor * lm)
            res.n_floored += int(np.sum(v < v_floor * lm))
            res.V[q] = 1.0 / fl
    else:
        raise ValueError(mode)
    return res


def merge(psiL, V, psiR, phys_q):
    """Psi'[a, s3, s4, b] = sum_alpha psiL[a, s3, alpha] V[alpha] psiR[alpha, s4, b]
    (Eq. eqn:merge)."""
    d = len(phys_q)
    out = {}
    for (qa, s3), XL in psiL.items():
        qm = qa + phys_q[s3]
        for s4 in range(d):
            XR = psiR.get((qm, s4))
            if XR is None:
                continue
            out[(qa, s3, s4)] = (XL * V[qm][None, :]) @ XR
    return out


def contract_two(X, Y, phys_q):
    """psi[a, s1, s2, b] = sum_alpha X[a, s1, alpha] Y[alpha, s2, b]."""
    d = len(phys_q)
    out = {}
    for (qa, s1), Xb in X.items():
        qm = qa + phys_q[s1]
        for s2 in range(d):
            Yb = Y.get((qm, s2))
            if Yb is not None:
                out[(qa, s1, s2)] = Xb @ Yb
    return out


# ----------------------------------------------------------------------------
# sweeps
# ----------------------------------------------------------------------------

@dataclass
class SweepParams:
    schedule: list                    # max m for each sweep
    n_warmup: int = 0                 # leading serial sweeps (Sec. II warm-up)
    n_regions: int = 1
    dav: DavidsonParams = field(default_factory=lambda: DavidsonParams(4, 1e-8, 8))
    dav_shared: DavidsonParams = field(default_factory=lambda: DavidsonParams(40, 1e-10, 8))
    cutoff: float = 1e-12
    eps: float = 1e-4
    region_order: str = "forward"     # order regions are visited between merges


class State:
    """MPS + MPO + environments.  bonds[b] is the sector list of bond b
    (between sites b-1 and b); L[b], R[b] are the environments living on bond b;
    V[b] is the inverse-singular-value vector stored on shared bond b."""

    def __init__(self, mpo, bonds, sites, q_target):
        self.mpo = mpo
        self.N = mpo.N
        self.phys_q = mpo.phys_q
        self.q_target = q_target
        self.bonds = list(bonds)
        self.sites = list(sites)
        self.L = [None] * (self.N + 1)
        self.R = [None] * (self.N + 1)
        self.V = {}
        self.log = []

    def dl(self, b):
        return self.mpo.deltas[b]


def canonicalize_right(st):
    """Bring the MPS to right-canonical form with the centre on site 0 by
    single-site SVDs from the right (no truncation beyond exact zeros), then
    normalise and build every right environment."""
    pq = st.phys_q
    d = len(pq)
    for i in range(st.N - 1, 0, -1):
        bl, br = st.bonds[i], st.bonds[i + 1]
        newB, G, newdims = {}, {}, {}
        for qa in bl.qs:
            ss = [s for s in range(d) if br.has(qa + pq[s])]
            if not ss:
                continue
            M = np.hstack([st.sites[i][(qa, s)] for s in ss])
            U, lam, Vt = svd_gesvd(M)
            r = int(np.sum(lam > 1e-14 * lam[0])) if lam.size and lam[0] > 0 else 0
            if r == 0:
                continue
            c0 = 0
            for s in ss:
                w = br.dim(qa + pq[s])
                newB[(qa, s)] = Vt[:r, c0:c0 + w].copy()
                c0 += w
            G[qa] = U[:, :r] * lam[None, :r]
            newdims[qa] = r
        st.sites[i] = newB
        st.bonds[i] = Bond(newdims)
        prev = {}
        for (qa, s), Xb in st.sites[i - 1].items():
            qb = qa + pq[s]
            if qb in G:
                prev[(qa, s)] = Xb @ G[qb]
        st.sites[i - 1] = prev
    nrm = norm(st.sites[0])
    st.sites[0] = {k: v / nrm for k, v in st.sites[0].items()}
    st.L[0] = left_boundary()
    st.R[st.N] = right_boundary(st.q_target)
    for i in range(st.N - 1, 0, -1):
        st.R[i] = update_R(st.R[i + 1], st.sites[i], st.mpo.W[i], pq, st.dl(i), st.dl(i + 1))


def _solve_bond(st, i, psi, dav):
    """Davidson on the two-site wavefunction at sites (i, i+1)."""
    pq = st.phys_q
    bl, br = st.bonds[i], st.bonds[i + 2]
    keys = two_site_keys(bl, br, pq)
    shapes = [two_site_shape(k, bl, br, pq) for k in keys]
    W1, W2 = st.mpo.W[i], st.mpo.W[i + 1]
    dl, dr = st.dl(i), st.dl(i + 2)
    Lb, Rb = st.L[i], st.R[i + 2]

    def mv(v):
        return flatten(heff_apply(Lb, Rb, W1, W2, unflatten(v, keys, shapes), bl, br, pq, dl, dr), keys, shapes)

    diag = flatten(heff_diag(Lb, Rb, W1, W2, bl, br, pq, dl, dr), keys, shapes)
    x0 = flatten(psi, keys, shapes)
    E, x, rn, nmv = davidson(mv, x0, diag, dav)
    return E, unflatten(x, keys, shapes), rn, nmv


def _store(st, i, res, mode):
    pq = st.phys_q
    st.bonds[i + 1] = res.bond
    if mode == "right":
        st.sites[i], st.sites[i + 1] = res.A, res.center
        st.L[i + 1] = update_L(st.L[i], res.A, st.mpo.W[i], pq, st.dl(i), st.dl(i + 1))
    elif mode == "left":
        st.sites[i], st.sites[i + 1] = res.center, res.B
        st.R[i + 1] = update_R(st.R[i + 2], res.B, st.mpo.W[i + 1], pq, st.dl(i + 1), st.dl(i + 2))
    else:
        st.sites[i], st.sites[i + 1] = res.left, res.right
        st.V[i + 1] = res.V
        st.L[i + 1] = update_L(st.L[i], res.A, st.mpo.W[i], pq, st.dl(i), st.dl(i + 1))
        st.R[i + 1] = update_R(st.R[i + 2], res.B, st.mpo.W[i + 1], pq, st.dl(i + 1), st.dl(i + 2))


def optimize_bond(st, i, mode, m, p, dav=None, psi=None, tag="bond"):
    """One two-site DMRG step at sites (i, i+1) (Sec. II)."""
    pq = st.phys_q
    if psi is None:
        psi = contract_two(st.sites[i], st.sites[i + 1], pq)
    E, psi, rn, nmv = _solve_bond(st, i, psi, dav or p.dav)
    res = svd_truncate(psi, st.bonds[i], st.bonds[i + 2], pq, m, mode, p.cutoff, p.eps)
    _store(st, i, res, mode)
    st.log.append(dict(kind=tag, site=i, E=E, resid=rn, nmv=nmv, trunc=res.discarded,
                       m=res.bond.total()))
    return E


def gauge_move(st, i, mode, m, p):
    """Move an orthogonality centre across bond i+1 by an SVD (no eigensolver)."""
    psi = contract_two(st.sites[i], st.sites[i + 1], st.phys_q)
    res = svd_truncate(psi, st.bonds[i], st.bonds[i + 2], st.phys_q, m, mode, p.cutoff, p.eps)
    _store(st, i, res, mode)


def serial_sweep(st, m, p):
    """Standard finite two-site sweep: bonds 0..N-2 moving right, then back."""
    for i in range(st.N - 1):
        optimize_bond(st, i, "right", m, p)
    for i in range(st.N - 2, -1, -1):
        optimize_bond(st, i, "left", m, p)


def regions_of(N, n):
    size = N // n
    assert size >= 2 and size * n == N, "regions must hold >= 2 sites and tile the chain"
    return [(r * size, (r + 1) * size - 1) for r in range(n)]


def split_regions(st, regions, m, p):
    """From a state with its centre on site 0, insert V = Lambda^{-1} on every
    shared bond (Eqs. eqn:inverse, eqn:isvd) and place the centres in the
    staggered start positions of Fig. 4: odd regions (1-based) at their left
    end, even regions at their right end.  Pure gauge moves, no eigensolver."""
    n = len(regions)
    for r, (lo, hi) in enumerate(regions):
        for i in range(lo, hi):
            gauge_move(st, i, "right", m, p)
        if r < n - 1:
            psi = contract_two(st.sites[hi], st.sites[hi + 1], st.phys_q)
            res = svd_truncate(psi, st.bonds[hi], st.bonds[hi + 2], st.phys_q, m, "split", p.cutoff, p.eps)
            _store(st, hi, res, "split")
    for r, (lo, hi) in enumerate(regions):
        if r % 2 == 0:
            for i in range(hi - 1, lo - 1, -1):
                gauge_move(st, i, "left", m, p)


def prediction_infidelity(pred, psi):
    """Fig. 3's measure of the merge prediction: 1 - |<Psi'|Psi>| / (|Psi'| |Psi|)
    for the merged state Psi' = psi_L V psi_R and the optimised Psi."""
    ov = sum(float(np.sum(pred[k] * psi[k])) for k in pred if k in psi)
    den = norm(pred) * norm(psi)
    return max(0.0, 1.0 - abs(ov) / den) if den > 0 else 1.0


def merge_shared(st, j, m, p):
    """Merge at the shared bond between sites j and j+1 with the stored V
    (Eq. eqn:merge), optimise the merged state, and split it again."""
    pq = st.phys_q
    psi = merge(st.sites[j], st.V[j + 1], st.sites[j + 1], pq)
    nrm = norm(psi)
    psi = {k: v / nrm for k, v in psi.items()}
    pred = psi
    E, psi, rn, nmv = _solve_bond(st, j, psi, p.dav_shared)
    infid = prediction_infidelity(pred, psi)
    res = svd_truncate(psi, st.bonds[j], st.bonds[j + 2], pq, m, "split", p.cutoff, p.eps)
    _store(st, j, res, "split")
    st.log.append(dict(kind="merge", site=j, E=E, resid=rn, nmv=nmv, trunc=res.discarded,
                       m=res.bond.total(), floored=res.n_floored, infidelity=infid))
    return E


def parallel_sweep(st, regions, m, p):
    """One full parallel sweep (Fig. 4): half-sweep A (odd regions move right,
    even regions move left), merges at shared bonds 1|2, 3|4, ...; half-sweep
    B (all regions move back), merges at 2|3, 4|5, ...  With one region this
    is exactly the serial sweep."""
    n = len(regions)
    order = list(range(n)) if p.region_order == "forward" else list(range(n))[::-1]
    for half in (0, 1):
        for r in order:
            lo, hi = regions[r]
            right = (r % 2 == 0) == (half == 0)
            if right:
                for i in range(lo, hi):
                    optimize_bond(st, i, "right", m, p)
            else:
                for i in range(hi - 1, lo - 1, -1):
                    optimize_bond(st, i, "left", m, p)
        for r in range(half, n - 1, 2):
            merge_shared(st, regions[r][1], m, p)


def expectation(st, Ws, deltas):
    """<Psi|O|Psi> of the full MPS (site tensors with V on shared bonds)."""
    pq = st.phys_q
    E = left_boundary()
    for i in range(st.N):
        E = update_L(E, st.sites[i], Ws[i], pq, deltas[i], deltas[i + 1])
        if (i + 1) in st.V:
            V = st.V[i + 1]
            E = {(q, w): V[q][:, None] * blk * V[q - deltas[i + 1][w]][None, :] for (q, w), blk in E.items()}
    return float(E[(st.q_target, 0)][0, 0])


def energy(st):
    """<Psi|H|Psi>/<Psi|Psi> of the whole MPS, contracted site by site."""
    d = len(st.phys_q)
    ident = [np.eye(d).reshape(1, d, d, 1)] * st.N
    zeros = [np.zeros(1, dtype=np.int64)] * (st.N + 1)
    return expectation(st, st.mpo.W, st.mpo.deltas) / expectation(st, ident, zeros)


def run_dmrg(mpo, bonds, sites, q_target, p):
    """Warm-up serial sweeps, split, then parallel sweeps; returns the state
    and the end-of-sweep energies."""
    st = State(mpo, [Bond(b) if not isinstance(b, Bond) else b for b in bonds],
               [dict(s) for s in sites], q_target)
    canonicalize_right(st)
    energies = []
    regions = regions_of(st.N, p.n_regions)
    for k, m in enumerate(p.schedule):
        if k < p.n_warmup or p.n_regions == 1:
            serial_sweep(st, m, p)
        else:
            if k == p.n_warmup:
                split_regions(st, regions, m, p)
            parallel_sweep(st, regions, m, p)
        energies.append(energy(st))
    return st, energies
