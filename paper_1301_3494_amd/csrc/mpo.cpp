// MPO builder (host): lattice Hamiltonians of Sec. III as a finite-state
// machine over term prefixes.
//
// Spin-1/2 basis ordered by charge q = 2 S^z: index 0 = down, 1 = up.
// Sites of an Lx x Ly cylinder (open x, periodic y) are numbered column by
// column in a snake.  A term is coef * prod_k op_k(site_k) with increasing
// sites.  At MPO bond b (between sites b-1 and b) the channels are 'start'
// (some term begins at a site >= b), every distinct prefix (the operators a
// term has placed on sites < b, for terms straddling the bond; shared by all
// terms with that prefix, ordered lexicographically by (site, operator)),
// and 'done' (some term ended before b).  A term's coupling is carried by
// its last operator.
#include "internal.hpp"

#include <cmath>
#include <map>
#include <set>
#include <tuple>

using namespace pdmrg;

namespace {

enum Op { I = 0, SZ = 1, SP = 2, SM = 3, SX = 4 };

struct Term {
    double coef;
    std::vector<std::pair<int, int>> f;   // (site, op), sites increasing
};

const double kOps[5][2][2] = {
    {{1, 0}, {0, 1}},          // I
    {{-0.5, 0}, {0, 0.5}},     // Sz
    {{0, 0}, {1, 0}},          // S+ = |up><down|
    {{0, 1}, {0, 0}},          // S- = |down><up|
    {{0, 0.5}, {0.5, 0}},      // Sx
};
const int kOpCharge[5] = {0, 0, 2, -2, 0};

int snake(int x, int y, int Ly) { return lattice_snake(x, y, Ly); }

std::vector<std::pair<int, int>> square_bonds(int Lx, int Ly) {
    std::set<std::pair<int, int>> b;
    for (int x = 0; x < Lx; ++x)
        for (int y = 0; y < Ly; ++y) {
            if (Ly > 2 || (Ly == 2 && y == 0)) {
                int a = snake(x, y, Ly), c = snake(x, (y + 1) % Ly, Ly);
                b.insert({std::min(a, c), std::max(a, c)});
            }
            if (x + 1 < Lx) {
                int a = snake(x, y, Ly), c = snake(x + 1, y, Ly);
                b.insert({std::min(a, c), std::max(a, c)});
            }
        }
    return {b.begin(), b.end()};
}

std::vector<std::pair<int, int>> triangular_bonds(int Lx, int Ly) {
    auto sq = square_bonds(Lx, Ly);
    std::set<std::pair<int, int>> b(sq.begin(), sq.end());
    if (Ly >= 2)
        for (int x = 0; x + 1 < Lx; ++x)
            for (int y = 0; y < Ly; ++y) {
                int a = snake(x, y, Ly), c = snake(x + 1, (y - 1 + Ly) % Ly, Ly);
                b.insert({std::min(a, c), std::max(a, c)});
            }
    return {b.begin(), b.end()};
}

Term make(double c, std::vector<std::pair<int, int>> f) {
    std::sort(f.begin(), f.end());
    for (size_t k = 1; k < f.size(); ++k)
        PD_REQUIRE(f[k].first != f[k - 1].first, PDMRG_EINVAL, "mpo_build: repeated site in a term");
    return Term{c, f};
}

// S_a . S_b = Sz Sz + (S+ S- + S- S+)/2
const std::tuple<double, int, int> kDot[3] = {{1.0, SZ, SZ}, {0.5, SP, SM}, {0.5, SM, SP}};

void add_xxz(std::vector<Term> &t, const std::vector<std::pair<int, int>> &bonds, double J, double Delta) {
    for (auto [i, j] : bonds) {
        t.push_back(make(J * Delta, {{i, SZ}, {j, SZ}}));
        t.push_back(make(0.5 * J, {{i, SP}, {j, SM}}));
        t.push_back(make(0.5 * J, {{i, SM}, {j, SP}}));
    }
}

}  // namespace

namespace {
// The MPO of a lattice model at the given couplings (throws on bad input).
std::unique_ptr<pdmrg_mpo> build_model(int lattice, int Lx, int Ly, const std::vector<double> &cpl) {
    {
        const double *couplings = cpl.data();
        const int ncouplings = (int)cpl.size();
        PD_REQUIRE(ncouplings >= 2 && Lx >= 1, PDMRG_EINVAL, "mpo_build: bad arguments");
        const double c0 = couplings[0], c1 = couplings[1];
        std::vector<Term> terms;
        int N = 0;
        std::vector<int> phys_q = {-1, 1};
        switch (lattice) {
            case 0:   // open chain, {J, Delta}
                N = Lx;
                {
                    std::vector<std::pair<int, int>> b;
                    for (int i = 0; i + 1 < N; ++i) b.push_back({i, i + 1});
                    add_xxz(terms, b, c0, c1);
                }
                break;
            case 1:   // square cylinder, {J, Delta}
                N = Lx * Ly;
                add_xxz(terms, square_bonds(Lx, Ly), c0, c1);
                break;
            case 2: { // triangular cylinder, {J, Delta} or {J, Delta, h}
                N = Lx * Ly;
                add_xxz(terms, triangular_bonds(Lx, Ly), c0, c1);
                const double h = ncouplings >= 3 ? couplings[2] : 0.0;
                if (h != 0.0) {
                    // pinning field -h S^z on the sites of sublattice (x - y) mod 3 = 0 of
                    // the two open edge columns (a 3-colouring of the bond set: needs Ly % 3 == 0)
                    PD_REQUIRE(Ly % 3 == 0 && Lx >= 2, PDMRG_EINVAL, "mpo_build: triangular pinning needs Ly % 3 == 0");
                    for (int x : {0, Lx - 1})
                        for (int y = 0; y < Ly; ++y)
                            if (tri_sublattice(x, y) == 0) terms.push_back(make(-h, {{snake(x, y, Ly), SZ}}));
                }
                break;
            }
            case 3: { // J-Q2 cylinder, {J, Q}
                PD_REQUIRE(Ly >= 3, PDMRG_EINVAL, "mpo_build: J-Q2 needs Ly >= 3");
                N = Lx * Ly;
                const double J = c0, Q = c1;
                add_xxz(terms, square_bonds(Lx, Ly), J, 1.0);
                double cst = 0.0;
                for (int x = 0; x + 1 < Lx; ++x)
                    for (int y = 0; y < Ly; ++y) {
                        const int y1 = (y + 1) % Ly;
                        const int p00 = snake(x, y, Ly), p10 = snake(x + 1, y, Ly);
                        const int p01 = snake(x, y1, Ly), p11 = snake(x + 1, y1, Ly);
                        const std::pair<int, int> pairs[2][2] = {{{p00, p10}, {p01, p11}},
                                                                 {{p00, p01}, {p10, p11}}};
                        for (auto &pr : pairs) {
                            auto [a, b] = pr[0];
                            auto [c, d] = pr[1];
                            for (auto [ca, oa, ob] : kDot)
                                for (auto [cc, oc, od] : kDot)
                                    terms.push_back(make(-Q * ca * cc, {{a, oa}, {b, ob}, {c, oc}, {d, od}}));
                            for (auto [x0, x1] : {pr[0], pr[1]})
                                for (auto [cx, o0, o1] : kDot) terms.push_back(make(0.25 * Q * cx, {{x0, o0}, {x1, o1}}));
                            cst += -Q / 16.0;
                        }
                    }
                const double pin = ncouplings >= 3 ? couplings[2] : 0.0;
                if (pin != 0.0) {
                    // edge pinning: pin (Q/4)(S_r . S_{r+y} - 1/4) on every vertical bond
                    // of the two open edge columns
                    for (int x : {0, Lx - 1})
                        for (int y = 0; y < Ly; ++y) {
                            const int a = snake(x, y, Ly), b = snake(x, (y + 1) % Ly, Ly);
                            for (auto [cx, o0, o1] : kDot)
                                terms.push_back(make(pin * 0.25 * Q * cx, {{std::min(a, b), o0}, {std::max(a, b), o1}}));
                            cst += -pin * Q / 16.0;
                        }
                }
                terms.push_back(make(cst, {{0, I}}));
                break;
            }
            case 4:   // transverse-field Ising chain, {J, h}; no symmetry
                N = Lx;
                phys_q = {0, 0};
                for (int i = 0; i + 1 < N; ++i) terms.push_back(make(-4.0 * c0, {{i, SZ}, {i + 1, SZ}}));
                for (int i = 0; i < N; ++i) terms.push_back(make(-2.0 * c1, {{i, SX}}));
                break;
            case 5:   // open S = 1 chain, {J, Delta}; local states q = 2 S^z = -2, 0, 2
                N = Lx;
                phys_q = {-2, 0, 2};
                {
                    std::vector<std::pair<int, int>> b;
                    for (int i = 0; i + 1 < N; ++i) b.push_back({i, i + 1});
                    add_xxz(terms, b, c0, c1);
                }
                break;
            default:
                throw Error(PDMRG_EINVAL, "mpo_build: unknown lattice");
        }
        PD_REQUIRE(N >= 2, PDMRG_EINVAL, "mpo_build: need at least two sites");
        const int d = (int)phys_q.size();
        bool trivial = true;
        for (int q : phys_q) trivial = trivial && q == 0;
        // local operators <s|O|t> (row-major d x d): spin 1/2 (down, up) or spin 1 (m = -1, 0, 1)
        std::vector<std::vector<double>> ops(5);
        if (d == 2) {
            for (int o = 0; o < 5; ++o)
                for (int a = 0; a < 2; ++a)
                    for (int c = 0; c < 2; ++c) ops[o].push_back(kOps[o][a][c]);
        } else {
            const double r2 = std::sqrt(2.0);
            ops[I] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
            ops[SZ] = {-1, 0, 0, 0, 0, 0, 0, 0, 1};
            ops[SP] = {0, 0, 0, r2, 0, 0, 0, r2, 0};   // S+ |m> = sqrt(2) |m + 1>
            ops[SM] = {0, r2, 0, 0, 0, r2, 0, 0, 0};
            ops[SX] = {0, r2 / 2, 0, r2 / 2, 0, r2 / 2, 0, r2 / 2, 0};
        }

        // channel sets
        using Prefix = std::vector<std::pair<int, int>>;
        std::vector<std::vector<Prefix>> chans(N + 1);
        std::vector<char> has_start(N + 1, 0), has_done(N + 1, 0);
        for (int b = 0; b <= N; ++b) {
            std::set<Prefix> pre;
            for (const Term &t : terms) {
                const int fs = t.f.front().first, ls = t.f.back().first;
                if (fs >= b) has_start[b] = 1;
                if (ls < b) has_done[b] = 1;
                if (fs < b && b <= ls) {
                    Prefix p;
                    for (auto &f : t.f)
                        if (f.first < b) p.push_back(f);
                    pre.insert(p);
                }
            }
            chans[b].assign(pre.begin(), pre.end());
        }
        // channel index: start = 0 if present, prefixes, done last
        auto D = [&](int b) { return has_start[b] + (int)chans[b].size() + has_done[b]; };
        auto idx_start = [&](int b) { return has_start[b] ? 0 : -1; };
        auto idx_done = [&](int b) { return has_done[b] ? D(b) - 1 : -1; };
        auto idx_pre = [&](int b, const Prefix &p) {
            auto it = std::lower_bound(chans[b].begin(), chans[b].end(), p);
            PD_REQUIRE(it != chans[b].end() && *it == p, PDMRG_EINVAL, "mpo_build: missing prefix channel");
            return has_start[b] + (int)(it - chans[b].begin());
        };
        auto pre_charge = [&](const Prefix &p) {
            int c = 0;
            for (auto &f : p) c += trivial ? 0 : kOpCharge[f.second];
            return c;
        };

        auto m = std::make_unique<pdmrg_mpo>();
        m->N = N;
        m->d = d;
        m->phys_q = phys_q;
        m->W.resize(N);
        std::vector<std::vector<int>> deltas(N + 1);
        for (int b = 0; b <= N; ++b) {
            deltas[b].assign(D(b), 0);
            for (size_t k = 0; k < chans[b].size(); ++k) deltas[b][has_start[b] + k] = pre_charge(chans[b][k]);
        }
        for (int i = 0; i < N; ++i) {
            MpoSite &W = m->W[i];
            W.Dl = D(i);
            W.Dr = D(i + 1);
            W.d = d;
            W.dl = deltas[i];
            W.dr = deltas[i + 1];
            W.W.assign((size_t)W.Dl * d * d * W.Dr, 0.0);
        }
        auto put = [&](int i, int wl, int wr, int op, double c, bool add) {
            PD_REQUIRE(wl >= 0 && wr >= 0, PDMRG_EINVAL, "mpo_build: missing channel");
            MpoSite &W = m->W[i];
            for (int s = 0; s < d; ++s)
                for (int t = 0; t < d; ++t) {
                    double &e = W.W[(((size_t)wl * d + s) * d + t) * W.Dr + wr];
                    const double v = c * ops[op][(size_t)s * d + t];
                    if (add) e += v;
                    else {
                        PD_REQUIRE(e == 0.0 || e == v, PDMRG_EINVAL, "mpo_build: inconsistent shared transition");
                        e = v;
                    }
                }
        };
        for (int i = 0; i < N; ++i) {
            if (idx_start(i) >= 0 && idx_start(i + 1) >= 0) put(i, idx_start(i), idx_start(i + 1), I, 1.0, false);
            if (idx_done(i) >= 0) put(i, idx_done(i), idx_done(i + 1), I, 1.0, false);
        }
        for (const Term &t : terms) {
            const int k = (int)t.f.size();
            if (k == 1) {
                const int s = t.f[0].first;
                put(s, idx_start(s), idx_done(s + 1), t.f[0].second, t.coef, true);
                continue;
            }
            auto prefix = [&](int j) { return Prefix(t.f.begin(), t.f.begin() + j + 1); };
            for (int i = t.f.front().first; i <= t.f.back().first; ++i) {
                int pos = -1, before = 0;   // index of site i in the term; factors on sites < i
                for (int q = 0; q < k; ++q) {
                    if (t.f[q].first == i) pos = q;
                    if (t.f[q].first < i) ++before;
                }
                if (pos == 0) {
                    put(i, idx_start(i), idx_pre(i + 1, prefix(0)), t.f[0].second, 1.0, false);
                } else if (pos == k - 1) {
                    put(i, idx_pre(i, prefix(pos - 1)), idx_done(i + 1), t.f[pos].second, t.coef, true);
                } else if (pos > 0) {
                    put(i, idx_pre(i, prefix(pos - 1)), idx_pre(i + 1, prefix(pos)), t.f[pos].second, 1.0, false);
                } else {
                    put(i, idx_pre(i, prefix(before - 1)), idx_pre(i + 1, prefix(before - 1)), I, 1.0, false);
                }
            }
        }
        return m;
    }
}

bool same_structure(const pdmrg_mpo &a, const pdmrg_mpo &b) {
    if (a.N != b.N || a.d != b.d) return false;
    for (int i = 0; i < a.N; ++i)
        if (a.W[i].Dl != b.W[i].Dl || a.W[i].Dr != b.W[i].Dr || a.W[i].dl != b.W[i].dl || a.W[i].dr != b.W[i].dr)
            return false;
    return true;
}
}  // namespace

extern "C" int mpo_build(int lattice, int Lx, int Ly, const double *couplings, int ncouplings, pdmrg_mpo **out) {
    try {
        PD_REQUIRE(out && couplings && ncouplings >= 2, PDMRG_EINVAL, "mpo_build: bad arguments");
        const std::vector<double> c(couplings, couplings + ncouplings);
        auto m = build_model(lattice, Lx, Ly, c);
        // coefficient derivatives dW/dtheta_k: every coefficient of these
        // models is affine in each coupling with the others held fixed, so
        // W(theta + e_k) - W(theta) is the derivative (not kept if the
        // channel structure changed)
        m->dW.assign(ncouplings, std::vector<double>());
        for (int k = 0; k < ncouplings; ++k) {
            std::vector<double> ck = c;
            ck[k] += 1.0;
            auto up = build_model(lattice, Lx, Ly, ck);
            if (!same_structure(*m, *up)) continue;
            std::vector<double> &d = m->dW[k];
            for (int i = 0; i < m->N; ++i)
                for (size_t e = 0; e < m->W[i].W.size(); ++e) d.push_back(up->W[i].W[e] - m->W[i].W[e]);
        }
        *out = m.release();
        return PDMRG_OK;
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return PDMRG_EINVAL;
    }
}
