"""Matrix-product-operator builder (oracle; test infrastructure only).

The paper works with "projected operators" (Sec. II) without fixing a form;
here the Hamiltonian is an MPO W_0 ... W_{N-1}, W_i[wl, s, s', wr] being the
operator matrix element <s|O|s'> for the channel transition wl -> wr.

Construction: a finite-state machine over term prefixes.  At the bond b
(between sites b-1 and b) the channels are
  'start'  -- nothing placed yet (exists if some term starts at a site >= b),
  prefixes -- the operators a term has placed on sites < b, for every term
              whose first site is < b and last site is >= b; terms with the
              same prefix share the channel,
  'done'   -- a complete term (exists if some term ends at a site < b).
The coefficient of a term sits on its last operator.  Channel charge
delta = total charge q = 2 S^z that the channel's operators have added.
"""
import numpy as np


def op_charge(op, phys_q):
    """Charge delta = q_s - q_s' shared by all nonzero entries <s|op|s'>."""
    nz = np.argwhere(np.abs(op) > 0)
    deltas = {phys_q[s] - phys_q[t] for s, t in nz}
    assert len(deltas) <= 1, "operator does not carry a definite charge"
    return deltas.pop() if deltas else 0


class MPO:
    def __init__(self, W, channels, deltas, phys_q):
        self.W = W                  # list of N arrays [Dl, d, d, Dr]
        self.channels = channels    # list of N+1 channel-key lists
        self.deltas = deltas        # list of N+1 int arrays
        self.phys_q = tuple(phys_q)
        self.N = len(W)
        self.d = len(phys_q)

    def D(self, b):
        return len(self.channels[b])


def build_mpo(terms, N, ops, phys_q):
    d = len(phys_q)
    first = [min(s for s, _ in f) for _, f in terms]
    last = [max(s for s, _ in f) for _, f in terms]
    channels = []
    for b in range(N + 1):
        ch = []
        if any(fs >= b for fs in first):
            ch.append(("start",))
        prefixes = set()
        for (coef, factors), fs, ls in zip(terms, first, last):
            if fs < b <= ls:
                prefixes.add(tuple((s, o) for s, o in factors if s < b))
        ch += [("p",) + p for p in sorted(prefixes)]
        if any(ls < b for ls in last):
            ch.append(("done",))
        channels.append(ch)
    index = [{c: k for k, c in enumerate(ch)} for ch in channels]

    def charge(key):
        if key[0] != "p":
            return 0
        return sum(op_charge(ops[o], phys_q) for _, o in key[1:])

    deltas = [np.array([charge(c) for c in ch], dtype=np.int64) for ch in channels]
    W = [np.zeros((len(channels[i]), d, d, len(channels[i + 1]))) for i in range(N)]

    def put(i, wl, wr, mat, add=False):
        a, b = index[i].get(wl), index[i + 1].get(wr)
        assert a is not None and b is not None, (i, wl, wr)
        if add:
            W[i][a, :, :, b] += mat
        else:
            cur = W[i][a, :, :, b]
            assert not np.any(cur) or np.array_equal(cur, mat), "inconsistent shared transition"
            W[i][a, :, :, b] = mat

    eye = np.eye(d)
    for i in range(N):
        if ("start",) in index[i] and ("start",) in index[i + 1]:
            put(i, ("start",), ("start",), eye)
        if ("done",) in index[i]:
            put(i, ("done",), ("done",), eye)
    for coef, factors in terms:
        sites = [s for s, _ in factors]
        if len(factors) == 1:
            s, o = factors[0]
            put(s, ("start",), ("done",), coef * ops[o], add=True)
            continue
        prefix = lambda j: ("p",) + tuple(factors[:j + 1])   # ops on sites s_0..s_j
        for i in range(sites[0], sites[-1] + 1):
            if i in sites:
                j = sites.index(i)
                o = ops[factors[j][1]]
                if j == 0:
                    put(i, ("start",), prefix(0), o)
                elif j == len(factors) - 1:
                    put(i, prefix(j - 1), ("done",), coef * o, add=True)
                else:
                    put(i, prefix(j - 1), prefix(j), o)
            else:
                j = max(k for k, s in enumerate(sites) if s < i)
                put(i, prefix(j), prefix(j), eye)
    return MPO(W, channels, deltas, phys_q)


def mpo_to_dense(mpo):
    """Contract W_0 ... W_{N-1} into the full d^N x d^N matrix (site 0 is the
    most significant index)."""
    T = mpo.W[0][0]                      # [d, d, D1]  (bond 0 has one channel)
    for i in range(1, mpo.N):
        W = mpo.W[i]
        T = np.einsum("xyw,wstv->xsytv", T, W)
        n = T.shape[0] * T.shape[1]
        T = T.reshape(n, n, W.shape[3])
    return T[:, :, 0]


def terms_to_dense(terms, N, ops):
    """Brute-force Kronecker sum of the terms (independent of the MPO)."""
    d = ops["I"].shape[0]
    H = np.zeros((d ** N, d ** N))
    for coef, factors in terms:
        f = dict(factors)
        M = np.ones((1, 1))
        for s in range(N):
            M = np.kron(M, ops[f[s]] if s in f else ops["I"])
        H += coef * M
    return H


def operator_schmidt_rank(H, N, d, cut, tol=1e-10):
    """Rank of H across the cut between sites cut-1 and cut."""
    T = H.reshape([d] * (2 * N))
    left = list(range(cut)) + [N + k for k in range(cut)]
    right = list(range(cut, N)) + [N + k for k in range(cut, N)]
    M = T.transpose(left + right).reshape(d ** (2 * cut), d ** (2 * (N - cut)))
    s = np.linalg.svd(M, compute_uv=False)
    return int(np.sum(s > tol * s[0]))
