// MPS state and the sweep driver (Sec. II, Fig. 4) on the device.
//
// Serial two-site sweep: bonds 0..N-2 moving right (A kept, centre Lambda B),
// then back (B kept, centre A Lambda).  Real-space parallel sweep over n
// contiguous regions: V = Lambda^{-1} is inserted on every shared bond
// (Eqs. eqn:inverse, eqn:isvd), odd regions start at their left end and even
// ones at their right end; half-sweep A (odd right, even left) is followed by
// merges at shared bonds 1|2, 3|4, ... (Psi' = psi_L V psi_R, Eq. eqn:merge,
// optimised and split again), half-sweep B by merges at 2|3, 4|5, ...  With
// one region this is exactly the serial sweep.  No information crosses
// regions between merges, so the regions of one half-sweep are independent.
#include "internal.hpp"
#include "svd.hpp"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <functional>

using namespace pdmrg;

struct pdmrg_mps {
    int N = 0, q_target = 0;
    Phys p;
    std::vector<Bond> bonds;                 // N + 1
    std::vector<DevBuf> sites;               // SITE layouts, FP64
    std::vector<DevBuf> L, R;                // environments on bonds 0..N
    // V = Lambda^{-1} per bond (bond order; host and device copies) where
    // hasV[b] is set.  Sized N + 1 once, so the concurrent jobs of a sweep
    // only assign the slots of their own bonds and never change the
    // containers themselves.
    std::vector<std::vector<double>> V;
    std::vector<DevBuf> Vd;
    std::vector<char> hasV;
    void clear_v() {
        for (auto &v : V) v.clear();
        for (auto &d : Vd) d = DevBuf();
        std::fill(hasV.begin(), hasV.end(), 0);
    }
    bool ready = false;                      // canonical form + environments
    int n_regions = 1;
    bool split = false;
    bool icanon = false;                     // inverse canonical gauge: V on every inner bond
    std::vector<std::pair<int, int>> regions;
};

namespace {

struct Driver {
    pdmrg_ctx *ctx;
    pdmrg_mps *m;
    const pdmrg_mpo *mpo;
    pdmrg_sweep_params prm{};
    pdmrg_sweep_report rep{};
    double t_heff = 0.0, t_svd = 0.0, t_env = 0.0;   // wall seconds per step kind
    bool envs = true;   // gauge moves update environments (off: no MPO needed)
    // Environment recompute stride k (>= 2: between passes only every k-th
    // bond's environments and the region boundaries are kept; the others are
    // rebuilt from the nearest kept one when a pass needs them; <= 1: every
    // environment is kept).
    int stride = 0;

    hipStream_t s() const { return ctx->stream; }
    const MpoSite &W(int i) const { return mpo->W[i]; }

    int64_t site_size(int i) const { return site_layout(m->bonds[i], m->bonds[i + 1], m->p).size; }

    // psi2 = site i . site i+1 (optionally with V on the middle bond)
    DevBuf contract(int i, const double *Vdev) {
        MergePlan mp;
        mp.build(m->bonds[i], m->bonds[i + 1], m->bonds[i + 2], m->p, s());
        DevBuf out(std::max<int64_t>(mp.X.size, 1) * sizeof(double));
        if (Vdev) {
            ctx->ws_merge.ensure(std::max<int64_t>(mp.SR.size, 1) * sizeof(double));
            mp.run(m->sites[i].as<double>(), Vdev, m->sites[i + 1].as<double>(), out.as<double>(),
                   ctx->ws_merge.as<double>(), s());
        } else {
            launch_fill(out.as<double>(), 0.0, mp.X.size, s());
            Slots sl{};
            sl.p[0] = m->sites[i].ptr;
            sl.p[1] = m->sites[i + 1].ptr;
            sl.p[2] = out.ptr;
            mp.g.launch(GemmPrec::F64, true, sl, s());
        }
        HIP_OK(hipStreamSynchronize(s()));
        return out;
    }

    // Region boundaries: their environments are always kept (a region never
    // reaches past them for a recompute).
    bool boundary_L(int j) const {
        if (j == 0) return true;
        for (auto &r : m->regions) if (r.first == j) return true;
        return false;
    }
    bool boundary_R(int j) const {
        if (j == m->N) return true;
        for (auto &r : m->regions) if (r.second + 1 == j) return true;
        return false;
    }
    bool keep_L(int j) const { return stride <= 1 || j % stride == 0 || boundary_L(j); }
    bool keep_R(int j) const { return stride <= 1 || j % stride == 0 || boundary_R(j); }
    // Frees an environment the current pass leaves behind: `ckpt` keeps the
    // stride checkpoints (still valid for the next pass), otherwise only the
    // region boundaries stay.
    void drop_L(int j, bool ckpt) {
        if (stride <= 1 || j < 0 || j > m->N) return;
        if (ckpt ? keep_L(j) : boundary_L(j)) return;
        m->L[j] = DevBuf();
    }
    void drop_R(int j, bool ckpt) {
        if (stride <= 1 || j < 0 || j > m->N) return;
        if (ckpt ? keep_R(j) : boundary_R(j)) return;
        m->R[j] = DevBuf();
    }
    // L[i] / R[i] present: rebuilt from the nearest kept one towards the
    // outside of the pass (every environment on the way is kept until the
    // pass drops it).
    void ensure_L(int i) {
        if (m->L[i].ptr) return;
        int j = i - 1;
        while (j > 0 && !m->L[j].ptr) --j;
        PD_REQUIRE(m->L[j].ptr != nullptr, PDMRG_EINVAL, "sweep: no stored left environment to rebuild from");
        for (int t = j; t < i; ++t) env_L(t);
    }
    void ensure_R(int i) {
        if (m->R[i].ptr) return;
        int j = i + 1;
        while (j < m->N && !m->R[j].ptr) ++j;
        PD_REQUIRE(m->R[j].ptr != nullptr, PDMRG_EINVAL, "sweep: no stored right environment to rebuild from");
        for (int t = j - 1; t >= i; --t) env_R(t);
    }

    void env_L(int i) {   // L[i+1] from L[i] and site i
        ensure_L(i);
        const auto t0 = std::chrono::steady_clock::now();
        EnvPlan ep;
        ep.build(1, m->bonds[i], m->bonds[i + 1], m->p, W(i), s());
        DevBuf out(std::max<int64_t>(ep.Eout.size, 1) * sizeof(double));
        ctx->ws_env.ensure((size_t)(std::max<int64_t>(ep.nU1, 1) + std::max<int64_t>(ep.nU2, 1)) * sizeof(double));
        double *U1 = ctx->ws_env.as<double>();
        ep.run(GemmPrec::F64, m->L[i].ptr, m->sites[i].ptr, out.ptr, U1, U1 + std::max<int64_t>(ep.nU1, 1), s());
        HIP_OK(hipStreamSynchronize(s()));
        m->L[i + 1] = std::move(out);
        t_env += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void env_R(int i) {   // R[i] from R[i+1] and site i
        ensure_R(i + 1);
        const auto t0 = std::chrono::steady_clock::now();
        EnvPlan ep;
        ep.build(-1, m->bonds[i], m->bonds[i + 1], m->p, W(i), s());
        DevBuf out(std::max<int64_t>(ep.Eout.size, 1) * sizeof(double));
        ctx->ws_env.ensure((size_t)(std::max<int64_t>(ep.nU1, 1) + std::max<int64_t>(ep.nU2, 1)) * sizeof(double));
        double *U1 = ctx->ws_env.as<double>();
        ep.run(GemmPrec::F64, m->R[i + 1].ptr, m->sites[i].ptr, out.ptr, U1, U1 + std::max<int64_t>(ep.nU1, 1), s());
        HIP_OK(hipStreamSynchronize(s()));
        m->R[i] = std::move(out);
        t_env += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    DevBuf take(const DevBuf &src, int64_t n) {
        DevBuf d(std::max<int64_t>(n, 1) * sizeof(double));
        if (n) HIP_OK(hipMemcpyAsync(d.ptr, src.ptr, n * sizeof(double), hipMemcpyDeviceToDevice, s()));
        return d;
    }

    // store an SVD result at bond i+1 (sites i, i+1)
    void store(int i, SvdOut &r, int mode) {
        m->bonds[i + 1] = r.bnew;
        const int64_t na = site_layout(m->bonds[i], r.bnew, m->p).size;
        const int64_t nb = site_layout(r.bnew, m->bonds[i + 2], m->p).size;
        if (mode == PDMRG_ABSORB_RIGHT) {
            m->sites[i] = take(r.A, na);
            m->sites[i + 1] = take(r.right, nb);
            if (envs) env_L(i);
        } else if (mode == PDMRG_ABSORB_LEFT) {
            m->sites[i] = take(r.left, na);
            m->sites[i + 1] = take(r.B, nb);
            if (envs) env_R(i + 1);
        } else {
            // environments from the orthonormal factors A and B
            m->sites[i] = take(r.A, na);
            m->sites[i + 1] = take(r.B, nb);
            env_L(i);
            env_R(i + 1);
            m->sites[i] = take(r.left, na);
            m->sites[i + 1] = take(r.right, nb);
            m->V[i + 1] = r.V;
            m->Vd[i + 1] = DevBuf();
            upload(m->Vd[i + 1], r.V, s());
            m->hasV[i + 1] = 1;
            rep.n_floored += r.n_floored;
        }
        HIP_OK(hipStreamSynchronize(s()));
        rep.n_svd_unconverged += r.n_unconverged;
        rep.max_trunc = std::max(rep.max_trunc, r.discarded);
        rep.max_bond = std::max(rep.max_bond, r.bnew.total);
    }

    double solve(int i, DevBuf &psi, const pdmrg_dav_params &dav) {
        const Bond &bl = m->bonds[i], &br = m->bonds[i + 2];
        ensure_L(i);
        ensure_R(i + 2);
        const double *Ld = m->L[i].as<double>(), *Rd = m->R[i + 2].as<double>();
        pdmrg_heff op, op64;
        // bond shapes change from bond to bond and sweep to sweep: take tuned
        // plans from the cache, never time candidates here
        // FP64 operators read the environments in place; the low-precision
        // operator reuses the FP64 one's intermediates (the two alternate)
        const bool refine = prm.prec != PDMRG_F64 && prm.refine;
        if (refine) heff_build(ctx, &op64, bl, br, m->p, W(i), W(i + 1), Ld, Rd, PDMRG_F64, false, true);
        heff_build(ctx, &op, bl, br, m->p, W(i), W(i + 1), Ld, Rd, prm.prec, false, true, refine ? &op64 : nullptr);
        const auto t0 = std::chrono::steady_clock::now();
        DavResult r = davidson_run(ctx, &op, refine ? &op64 : nullptr, psi.as<double>(), dav);
        t_heff += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep.n_matvec += r.nmv;
        return r.energy;
    }

    void svd_timed(int i, const DevBuf &psi, int max_m, double cutoff, int mode, SvdOut &r) {
        const auto t0 = std::chrono::steady_clock::now();
        svd_truncate_run(ctx, m->bonds[i], m->bonds[i + 2], m->p, psi.as<double>(), max_m, cutoff, prm.eps, mode, r);
        t_svd += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    void optimize(int i, int mode, const pdmrg_dav_params &dav) {
        DevBuf psi = contract(i, nullptr);
        const double h0 = t_heff, s0 = t_svd;
        const double e = solve(i, psi, dav);
        SvdOut r;
        svd_timed(i, psi, prm.max_m, prm.cutoff, mode, r);
        store(i, r, mode);
        if (ctx->verbose)
            std::fprintf(stderr, "pdmrg: bond %d|%d m=%d E=%.12f davidson %.2fs svd %.2fs\n", i, i + 1,
                         m->bonds[i + 1].total, e, t_heff - h0, t_svd - s0),
                std::fflush(stderr);
    }

    void gauge_move(int i, int mode, int max_m, double cutoff) {
        DevBuf psi = contract(i, nullptr);
        const double s0 = t_svd;
        SvdOut r;
        svd_timed(i, psi, max_m, cutoff, mode, r);
        store(i, r, mode);
        if (ctx->verbose)
            std::fprintf(stderr, "pdmrg: gauge %d|%d m=%d svd %.2fs\n", i, i + 1, m->bonds[i + 1].total, t_svd - s0),
                std::fflush(stderr);
    }

    // 1 - |<a|b>| / (|a| |b|) of two device vectors (fixed-order reductions)
    double infidelity(const double *a, const double *b, int64_t n) {
        constexpr int kBlocks = 240;
        DevBuf part((size_t)kBlocks * 3 * sizeof(double)), out(3 * sizeof(double));
        const double *pairs[3][2] = {{a, b}, {a, a}, {b, b}};
        for (int k = 0; k < 3; ++k) {
            launch_multidot(pairs[k][0], n, 1, pairs[k][1], n, part.as<double>() + (size_t)k * kBlocks, kBlocks, s());
            launch_reduce_partials(part.as<double>() + (size_t)k * kBlocks, kBlocks, 1, out.as<double>() + k, 1, s());
        }
        double h[3];
        HIP_OK(hipMemcpyAsync(h, out.ptr, sizeof h, hipMemcpyDeviceToHost, s()));
        HIP_OK(hipStreamSynchronize(s()));
        const double den = std::sqrt(h[1] * h[2]);
        return den > 0.0 ? std::max(0.0, 1.0 - std::fabs(h[0]) / den) : 1.0;
    }

    void merge_shared(int j) {
        PD_REQUIRE(m->hasV[j + 1], PDMRG_EINVAL, "merge: no V on the shared bond");
        DevBuf psi = contract(j, m->Vd[j + 1].as<double>());
        // prediction fidelity of the merged state (Fig. 3): psi_L V psi_R
        // against the state the shared-bond eigensolver converges to
        const int64_t n = two_site_layout(m->bonds[j], m->bonds[j + 2], m->p).size;
        DevBuf pred = take(psi, n);
        const double e = solve(j, psi, prm.dav_shared);   // Davidson normalises its start vector
        const double inf = infidelity(pred.as<double>(), psi.as<double>(), n);
        rep.max_infidelity = std::max(rep.max_infidelity, inf);
        SvdOut r;
        svd_timed(j, psi, prm.max_m, prm.cutoff, PDMRG_SPLIT, r);
        store(j, r, PDMRG_SPLIT);
        if (ctx->verbose)
            std::fprintf(stderr, "pdmrg: merge %d|%d m=%d E=%.12f infidelity %.3e\n", j, j + 1, m->bonds[j + 1].total,
                         e, inf),
                std::fflush(stderr);
    }

    void init() {
        const int N = m->N;
        m->L.clear();
        m->R.clear();
        m->L.resize(N + 1);
        m->R.resize(N + 1);
        std::vector<double> one = {1.0};
        upload(m->L[0], one, s());
        upload(m->R[N], one, s());
        // right-canonical form with the centre on site 0, by two-site SVDs
        // from the right keeping every nonzero singular value
        for (int i = N - 2; i >= 0; --i) {
            gauge_move(i, PDMRG_ABSORB_LEFT, 1 << 30, 1e-14);
            drop_R(i + 2, true);
        }
        m->ready = true;
    }

    void split_regions() {
        const auto &rg = m->regions;
        const int n = (int)rg.size();
        for (int r = 0; r < n; ++r) {
            const int lo = rg[r].first, hi = rg[r].second;
            for (int i = lo; i < hi; ++i) gauge_move(i, PDMRG_ABSORB_RIGHT, prm.max_m, prm.cutoff);
            if (r < n - 1) gauge_move(hi, PDMRG_SPLIT, prm.max_m, prm.cutoff);
        }
        for (int r = 0; r < n; r += 2) {
            const int lo = rg[r].first, hi = rg[r].second;
            for (int i = hi - 1; i >= lo; --i) gauge_move(i, PDMRG_ABSORB_LEFT, prm.max_m, prm.cutoff);
        }
        m->split = true;
    }

    // One lockstep step over several bonds: one bond of every region, or the
    // shared bonds of a merge phase (Fig. 4).  The bonds share no sites or
    // environments.  The eigensolver runs per bond as independent jobs; the
    // truncated SVDs of all bonds share one batch (their sector blocks go
    // into the same Jacobi launches); then every bond stores its factors and
    // updates its environments as a job again.  The results equal those of
    // the bonds taken one at a time.
    struct Step {
        int i;         // bond between sites i and i + 1
        int mode;      // PDMRG_ABSORB_RIGHT, PDMRG_ABSORB_LEFT or PDMRG_SPLIT
        bool shared;   // merge at a shared bond: psi_L V psi_R, prediction fidelity
        bool right;    // direction of an interior step (which environments to drop)
    };
    void lockstep(const std::vector<Step> &steps) {
        const int n = (int)steps.size();
        std::vector<DevBuf> psi(n);
        std::vector<double> energy(n, 0.0), dav_s(n, 0.0);
        std::vector<std::function<void(Driver &)>> solve_jobs, store_jobs;
        for (int k = 0; k < n; ++k)
            solve_jobs.push_back([&, k](Driver &d) {
                const Step &st = steps[k];
                const double h0 = d.t_heff;
                if (st.shared) {
                    PD_REQUIRE(d.m->hasV[st.i + 1], PDMRG_EINVAL, "merge: no V on the shared bond");
                    psi[k] = d.contract(st.i, d.m->Vd[st.i + 1].as<double>());
                    // prediction fidelity of the merged state (Fig. 3): psi_L V
                    // psi_R against the state the shared-bond eigensolver reaches
                    const int64_t nx = two_site_layout(d.m->bonds[st.i], d.m->bonds[st.i + 2], d.m->p).size;
                    DevBuf pred = d.take(psi[k], nx);
                    energy[k] = d.solve(st.i, psi[k], d.prm.dav_shared);   // Davidson normalises its start
                    d.rep.max_infidelity =
                        std::max(d.rep.max_infidelity, d.infidelity(pred.as<double>(), psi[k].as<double>(), nx));
                } else {
                    psi[k] = d.contract(st.i, nullptr);
                    energy[k] = d.solve(st.i, psi[k], d.prm.dav);
                }
                dav_s[k] = d.t_heff - h0;
            });
        run_jobs(solve_jobs);
        std::vector<SvdProblem> probs;
        for (int k = 0; k < n; ++k)
            probs.push_back(SvdProblem{&m->bonds[steps[k].i], &m->bonds[steps[k].i + 2], &m->p, psi[k].as<double>(),
                                       prm.max_m, prm.cutoff, steps[k].mode});
        std::vector<SvdOut> outs;
        const auto t0 = std::chrono::steady_clock::now();
        svd_truncate_multi(ctx, probs, prm.eps, outs);
        const double svd_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        t_svd += svd_s;
        for (int k = 0; k < n; ++k)
            store_jobs.push_back([&, k](Driver &d) {
                const Step &st = steps[k];
                d.store(st.i, outs[k], st.mode);
                if (!st.shared) {
                    if (st.right) {
                        d.drop_L(st.i, true);
                        d.drop_R(st.i + 2, false);
                    } else {
                        d.drop_R(st.i + 2, true);
                        d.drop_L(st.i, false);
                    }
                }
                if (ctx->verbose)
                    std::fprintf(stderr, "pdmrg: bond %d|%d m=%d E=%.12f davidson %.2fs svd %.2fs (batch of %d)%s\n",
                                 st.i, st.i + 1, d.m->bonds[st.i + 1].total, energy[k], dav_s[k], svd_s, n,
                                 st.shared ? " merge" : ""),
                        std::fflush(stderr);
            });
        run_jobs(store_jobs);
    }

    // Context of region r for concurrent work: own non-blocking stream (default
    // priority) and work space, same device and tuning level.
    pdmrg_ctx *sub_ctx(int r) {
        while ((int)ctx->sub.size() <= r) {
            auto *c = new pdmrg_ctx();
            c->device = ctx->device;
            HIP_OK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
            c->owns_stream = true;
            ctx->sub.push_back(c);
        }
        ctx->sub[r]->autotune = ctx->autotune;
        ctx->sub[r]->graphs = ctx->graphs;
        ctx->sub[r]->verbose = ctx->verbose;
        ctx->sub[r]->svd_precond = ctx->svd_precond;
        return ctx->sub[r];
    }

    // Runs independent jobs (disjoint sites, bonds and environments): with
    // prm.concurrent, each on a worker thread of the context's pool with its
    // own stream and work space; else one after the other here.  Reports are
    // merged; the first error is rethrown.  Jobs only read the MPS containers
    // and assign the slots (sites, bonds, environments, V) of their own sites
    // and bonds.
    void run_jobs(const std::vector<std::function<void(Driver &)>> &jobs) {
        if (!prm.concurrent || jobs.size() <= 1) {
            for (auto &j : jobs) j(*this);
            return;
        }
        HIP_OK(hipStreamSynchronize(s()));
        const int n = (int)jobs.size();
        std::vector<Driver> ds;
        for (int k = 0; k < n; ++k) {
            Driver d{sub_ctx(k), m, mpo};
            d.prm = prm;
            d.envs = envs;
            d.stride = stride;
            ds.push_back(d);
        }
        if (!ctx->pool) ctx->pool.reset(new WorkerPool(ctx->device));
        std::vector<int> codes(n, 0);
        std::vector<std::string> msgs(n);
        const std::function<void(int)> body = [&](int k) {
            try {
                HIP_OK(hipSetDevice(ctx->device));
                jobs[k](ds[k]);
                HIP_OK(hipStreamSynchronize(ds[k].s()));
            } catch (const Error &e) {
                codes[k] = e.code;
                msgs[k] = e.what();
            } catch (const std::exception &e) {
                codes[k] = PDMRG_EINVAL;
                msgs[k] = e.what();
            }
        };
        ctx->pool->run(n, body);
        for (int k = 0; k < n; ++k) {
            const pdmrg_sweep_report &r = ds[k].rep;
            rep.n_matvec += r.n_matvec;
            rep.n_floored += r.n_floored;
            rep.max_trunc = std::max(rep.max_trunc, r.max_trunc);
            rep.max_bond = std::max(rep.max_bond, r.max_bond);
            rep.max_infidelity = std::max(rep.max_infidelity, r.max_infidelity);
            rep.n_svd_unconverged += r.n_svd_unconverged;
            t_heff += ds[k].t_heff;
            t_svd += ds[k].t_svd;
            t_env += ds[k].t_env;
        }
        for (int k = 0; k < n; ++k)
            if (codes[k] != 0) throw Error(codes[k], msgs[k]);
    }

    void parallel_sweep() {
        const auto rg = m->regions;
        const int n = (int)rg.size();
        if (prm.concurrent == 2) {
            lockstep_sweep();
            return;
        }
        for (int half = 0; half < 2; ++half) {
            std::vector<std::function<void(Driver &)>> jobs;
            for (int r = 0; r < n; ++r) {
                const int lo = rg[r].first, hi = rg[r].second;
                const bool right = (r % 2 == 0) == (half == 0);
                jobs.push_back([lo, hi, right](Driver &d) {
                    if (right)
                        for (int i = lo; i < hi; ++i) {
                            d.optimize(i, PDMRG_ABSORB_RIGHT, d.prm.dav);
                            d.drop_L(i, true);
                            d.drop_R(i + 2, false);
                        }
                    else
                        for (int i = hi - 1; i >= lo; --i) {
                            d.optimize(i, PDMRG_ABSORB_LEFT, d.prm.dav);
                            d.drop_R(i + 2, true);
                            d.drop_L(i, false);
                        }
                });
            }
            run_jobs(jobs);
            std::vector<std::function<void(Driver &)>> merges;
            for (int r = half; r < n - 1; r += 2) {
                const int j = rg[r].second;
                merges.push_back([j](Driver &d) { d.merge_shared(j); });
            }
            run_jobs(merges);
        }
    }

    // The staggered sweep of Fig. 4 with the regions in lockstep: step t
    // optimises bond t of every region (in its direction) and the merges of a
    // phase form one step, each step through lockstep().
    void lockstep_sweep() {
        const auto rg = m->regions;
        const int n = (int)rg.size();
        int len = 0;
        for (auto &r : rg) len = std::max(len, r.second - r.first);
        for (int half = 0; half < 2; ++half) {
            for (int t = 0; t < len; ++t) {
                std::vector<Step> steps;
                for (int r = 0; r < n; ++r) {
                    const int lo = rg[r].first, hi = rg[r].second;
                    if (t >= hi - lo) continue;
                    const bool right = (r % 2 == 0) == (half == 0);
                    steps.push_back(Step{right ? lo + t : hi - 1 - t, right ? PDMRG_ABSORB_RIGHT : PDMRG_ABSORB_LEFT,
                                         false, right});
                }
                lockstep(steps);
            }
            // merge phase: shared bonds 1|2, 3|4, ... then 2|3, 4|5, ...
            std::vector<Step> merges;
            for (int r = half; r < n - 1; r += 2) merges.push_back(Step{rg[r].second, PDMRG_SPLIT, true, false});
            if (!merges.empty()) lockstep(merges);
        }
    }

    // E[a, w, a'] *= V[a] V[a'] for a left environment E on bond b (ENV_L
    // layout El, channel charges dr): carries a transfer across a bond with V.
    void scale_env_v(DevBuf &E, const EnvLayout &El, const Bond &b, const std::vector<int> &dr, const double *V) {
        std::vector<CopyTask> ct;
        for (int j = 0; j < b.nsec(); ++j)
            for (int w = 0; w < El.D; ++w) {
                const int ro = El.rowo[(size_t)j * El.D + w];
                if (ro < 0) continue;
                const int k = b.find(b.q[j] + dr[w]);
                double *blk = E.as<double>() + El.base[j] + (int64_t)ro * b.dim[j];
                ct.push_back(CopyTask{blk, blk, V + b.off[k], V + b.off[j], b.dim[k], b.dim[j], b.dim[j], b.dim[j], 0, 0});
            }
        DevBuf d;
        upload(d, ct, s());
        int64_t mx = 0;
        for (auto &t : ct) mx = std::max<int64_t>(mx, (int64_t)t.rows * t.cols);
        launch_copies(d.as<CopyTask>(), (int)ct.size(), mx, s());
        HIP_OK(hipStreamSynchronize(s()));
    }

    // <Psi|O|Psi> of the whole MPS (V applied on shared bonds) by left transfer
    double expectation(bool identity) {
        const int N = m->N;
        DevBuf E;
        std::vector<double> one = {1.0};
        upload(E, one, s());
        std::vector<int> zero = {0};
        for (int i = 0; i < N; ++i) {
            MpoSite Wi;
            if (identity) {
                Wi.Dl = Wi.Dr = 1;
                Wi.d = m->p.d();
                Wi.W.assign((size_t)Wi.d * Wi.d, 0.0);
                for (int a = 0; a < Wi.d; ++a) Wi.W[(size_t)a * Wi.d + a] = 1.0;
                Wi.dl = zero;
                Wi.dr = zero;
            } else {
                Wi = W(i);
            }
            EnvPlan ep;
            ep.build(1, m->bonds[i], m->bonds[i + 1], m->p, Wi, s());
            DevBuf out(std::max<int64_t>(ep.Eout.size, 1) * sizeof(double));
            ctx->ws_env.ensure((size_t)(std::max<int64_t>(ep.nU1, 1) + std::max<int64_t>(ep.nU2, 1)) * sizeof(double));
            double *U1 = ctx->ws_env.as<double>();
            ep.run(GemmPrec::F64, E.ptr, m->sites[i].ptr, out.ptr, U1, U1 + std::max<int64_t>(ep.nU1, 1), s());
            if (m->split && m->hasV[i + 1]) scale_env_v(out, ep.Eout, m->bonds[i + 1], Wi.dr, m->Vd[i + 1].as<double>());
            HIP_OK(hipStreamSynchronize(s()));
            E = std::move(out);
        }
        double v = 0.0;
        HIP_OK(hipMemcpyAsync(&v, E.ptr, sizeof(double), hipMemcpyDeviceToHost, s()));
        HIP_OK(hipStreamSynchronize(s()));
        return v;
    }

    double energy() { return expectation(false) / expectation(true); }

    // Undo the region split: fold V into the left neighbour of every shared
    // bond (psi' = psi_L V psi_R re-split, dropping only singular values
    // below 1e-14 of the largest).
    void unsplit() {
        if (!m->split) return;
        for (int b = 1; b < m->N; ++b) {
            if (!m->hasV[b]) continue;
            const int j = b - 1;
            DevBuf psi = contract(j, m->Vd[b].as<double>());
            SvdOut r;
            svd_truncate_run(ctx, m->bonds[j], m->bonds[j + 2], m->p, psi.as<double>(), 1 << 30, 1e-14, prm.eps,
                             PDMRG_ABSORB_LEFT, r);
            m->bonds[j + 1] = r.bnew;
            m->sites[j] = take(r.left, site_layout(m->bonds[j], r.bnew, m->p).size);
            m->sites[j + 1] = take(r.B, site_layout(r.bnew, m->bonds[j + 2], m->p).size);
        }
        HIP_OK(hipStreamSynchronize(s()));
        m->clear_v();
        m->split = false;
        m->icanon = false;
        m->regions.clear();
        m->n_regions = 1;
    }

    // Inverse canonical gauge (Sec. IV): right-canonical form with the centre
    // on site 0, then the split of Eqs. eqn:inverse, eqn:isvd at bonds
    // 1..N-1 in order -- Theta = C_i B_{i+1} = (A Lambda) V (Lambda B), the
    // left factor stays as psi_i = Lambda_i Gamma_i Lambda_{i+1}, the right one
    // is the next centre.  Keeps every singular value >= cutoff * lambda_max.
    // Environments are not kept (the next sweep rebuilds them).
    int inverse_canonical(double cutoff) {
        unsplit();
        envs = false;
        init();
        int nfl = 0;
        for (int i = 0; i + 1 < m->N; ++i) {
            DevBuf psi = contract(i, nullptr);
            SvdOut r;
            svd_truncate_run(ctx, m->bonds[i], m->bonds[i + 2], m->p, psi.as<double>(), 1 << 30, cutoff, prm.eps,
                             PDMRG_SPLIT, r);
            m->bonds[i + 1] = r.bnew;
            m->sites[i] = take(r.left, site_layout(m->bonds[i], r.bnew, m->p).size);
            m->sites[i + 1] = take(r.right, site_layout(r.bnew, m->bonds[i + 2], m->p).size);
            m->V[i + 1] = r.V;
            m->Vd[i + 1] = DevBuf();
            upload(m->Vd[i + 1], r.V, s());
            m->hasV[i + 1] = 1;
            nfl += r.n_floored;
            HIP_OK(hipStreamSynchronize(s()));
        }
        m->L.clear();
        m->R.clear();
        m->L.resize(m->N + 1);
        m->R.resize(m->N + 1);
        m->split = true;
        m->icanon = true;
        m->ready = false;
        m->regions.clear();
        m->n_regions = 1;
        return nfl;
    }

    // <O_j> for every site j: one launch of column-segment products
    // <psi_j[:, s, :], psi_j[:, t, :]> over all sites and charge-conserving
    // (s, t) with O[s][t] != 0, weighted by O[s][t] on the host in task order.
    void expect_site(const std::vector<double> &op, double *out) {
        const int d = m->p.d();
        std::vector<SegDot> tasks;
        std::vector<int> site_of;
        std::vector<double> wt;
        for (int j = 0; j < m->N; ++j) {
            const SiteLayout S = site_layout(m->bonds[j], m->bonds[j + 1], m->p);
            for (int k = 0; k < m->bonds[j].nsec(); ++k)
                for (int a = 0; a < d; ++a)
                    for (int b = 0; b < d; ++b) {
                        const double c = op[(size_t)a * d + b];
                        const int wa = S.width[(size_t)k * d + a], wb = S.width[(size_t)k * d + b];
                        if (c == 0.0 || m->p.q[a] != m->p.q[b] || wa == 0 || wb == 0 || S.rows[k] == 0) continue;
                        tasks.push_back(SegDot{m->sites[j].as<double>() + S.base[k], S.cols[k], S.rows[k],
                                               S.colo[(size_t)k * d + a], S.colo[(size_t)k * d + b], wa, 0});
                        site_of.push_back(j);
                        wt.push_back(c);
                    }
        }
        for (int j = 0; j < m->N; ++j) out[j] = 0.0;
        if (tasks.empty()) return;
        std::vector<SegTile> tiles;
        std::vector<int32_t> t0, g_of;
        for (size_t t = 0; t < tasks.size(); ++t) {
            t0.push_back((int32_t)tiles.size());
            g_of.push_back((int32_t)t);
            for (int r0 = 0; r0 < tasks[t].rows; r0 += kSegRows) tiles.push_back(SegTile{(int32_t)t, r0});
        }
        t0.push_back((int32_t)tiles.size());
        DevBuf d_tasks, d_tiles, d_t0, d_g, partial, res;
        upload(d_tasks, tasks, s());
        upload(d_tiles, tiles, s());
        upload(d_t0, t0, s());
        upload(d_g, g_of, s());
        partial.ensure(tiles.size() * sizeof(double));
        res.ensure(tasks.size() * sizeof(double));
        launch_seg_dot_partials(d_tasks.as<SegDot>(), d_tiles.as<SegTile>(), (int)tiles.size(), partial.as<double>(),
                                s());
        launch_dot_reduce(partial.as<double>(), d_t0.as<int32_t>(), d_g.as<int32_t>(), (int)tasks.size(),
                          res.as<double>(), s());
        std::vector<double> h(tasks.size());
        HIP_OK(hipMemcpyAsync(h.data(), res.ptr, h.size() * sizeof(double), hipMemcpyDeviceToHost, s()));
        HIP_OK(hipStreamSynchronize(s()));
        for (size_t t = 0; t < tasks.size(); ++t) out[site_of[t]] += wt[t] * h[t];
    }

    // sum_t c_t <A_t(i) B_t(k)>, i < k, from the centres: identity on bond i,
    // left transfer through psi_i with W_i = [A_t], then through
    // B_j = V_j psi_j (V applied to the environment on bond j) with the
    // identity per channel, the last site with W_k = [c_t B_t], and the trace
    // on bond k+1.
    double correlator(int i, int k, const MpoSite &Wi, const MpoSite &Wm, const MpoSite &Wk) {
        const Bond &b0 = m->bonds[i];
        const EnvLayout E0 = env_l_layout(b0, std::vector<int>{0});
        DevBuf E(std::max<int64_t>(E0.size, 1) * sizeof(double));
        std::vector<SqBlock> sq;
        int mx = 0;
        for (int j = 0; j < b0.nsec(); ++j) {
            sq.push_back(SqBlock{E.as<double>() + E0.base[j], b0.dim[j], 0});
            mx = std::max(mx, b0.dim[j]);
        }
        DevBuf d_sq;
        upload(d_sq, sq, s());
        launch_set_identity(d_sq.as<SqBlock>(), (int)sq.size(), mx, s());
        HIP_OK(hipStreamSynchronize(s()));
        EnvLayout last;
        for (int j = i; j <= k; ++j) {
            const MpoSite &W = j == i ? Wi : (j < k ? Wm : Wk);
            EnvPlan ep;
            ep.build(1, m->bonds[j], m->bonds[j + 1], m->p, W, s());
            DevBuf out(std::max<int64_t>(ep.Eout.size, 1) * sizeof(double));
            ctx->ws_env.ensure((size_t)(std::max<int64_t>(ep.nU1, 1) + std::max<int64_t>(ep.nU2, 1)) * sizeof(double));
            double *U1 = ctx->ws_env.as<double>();
            ep.run(GemmPrec::F64, E.ptr, m->sites[j].ptr, out.ptr, U1, U1 + std::max<int64_t>(ep.nU1, 1), s());
            if (j < k) {
                PD_REQUIRE(m->hasV[j + 1], PDMRG_EINVAL, "correlator: no V on an inner bond");
                scale_env_v(out, ep.Eout, m->bonds[j + 1], W.dr, m->Vd[j + 1].as<double>());
            }
            HIP_OK(hipStreamSynchronize(s()));
            E = std::move(out);
            last = ep.Eout;
        }
        const Bond &bk = m->bonds[k + 1];
        std::vector<SqBlock> tr;
        for (int j = 0; j < bk.nsec(); ++j)
            if (last.rowo[j] >= 0) tr.push_back(SqBlock{E.as<double>() + last.base[j], bk.dim[j], 0});
        DevBuf d_tr, d_val;
        upload(d_tr, tr, s());
        d_val.ensure(sizeof(double));
        launch_trace_sum(d_tr.as<SqBlock>(), (int)tr.size(), d_val.as<double>(), s());
        double v = 0.0;
        HIP_OK(hipMemcpyAsync(&v, d_val.ptr, sizeof(double), hipMemcpyDeviceToHost, s()));
        HIP_OK(hipStreamSynchronize(s()));
        return v;
    }

    // Measurement sweep: right-canonical form with the centre on site 0, then
    // G_i at each centre i, moving the centre right by two-site SVDs that drop
    // only singular values below 1e-14 of the largest.  G_i is divided by
    // <Psi|Psi> (the centre's squared norm).
    void gradients(double *G, const std::vector<int64_t> &goff) {
        unsplit();
        init();
        for (int i = 0; i < m->N; ++i) {
            GradPlan gp;
            gp.build(m->bonds[i], m->bonds[i + 1], m->p, W(i), s());
            ensure_L(i);
            ensure_R(i + 1);
            grad_site_run(ctx, gp, m->L[i].as<double>(), m->sites[i].as<double>(), m->R[i + 1].as<double>(),
                          G + goff[i]);
            // G_i / <Psi|Psi>, the squared norm of the centre: a fixed-order
            // device reduction, then G scaled twice by 1/sqrt(norm^2)
            const int64_t n = site_layout(m->bonds[i], m->bonds[i + 1], m->p).size;
            constexpr int kBlocks = 240;
            DevBuf part((size_t)kBlocks * sizeof(double)), nrm(sizeof(double));
            launch_multidot(m->sites[i].as<double>(), n, 1, m->sites[i].as<double>(), n, part.as<double>(), kBlocks,
                            s());
            launch_reduce_partials(part.as<double>(), kBlocks, 1, nrm.as<double>(), 1, s());
            const int64_t gn = goff[i + 1] - goff[i];
            launch_scale_by_inv_sqrt(G + goff[i], nrm.as<double>(), G + goff[i], gn, s());
            launch_scale_by_inv_sqrt(G + goff[i], nrm.as<double>(), G + goff[i], gn, s());
            double nrm2 = 0.0;
            HIP_OK(hipMemcpyAsync(&nrm2, nrm.ptr, sizeof(double), hipMemcpyDeviceToHost, s()));
            HIP_OK(hipStreamSynchronize(s()));
            PD_REQUIRE(nrm2 > 0.0 && std::isfinite(nrm2), PDMRG_ENUMERIC, "grad_mpo: zero or non-finite state");
            if (i + 1 < m->N) gauge_move(i, PDMRG_ABSORB_RIGHT, 1 << 30, 1e-14);
            drop_L(i, false);
            drop_R(i + 1, false);
        }
        m->ready = false;   // centre now on the last site: the next sweep re-canonicalises
    }
};

// Charge q_s - q_t shared by every nonzero <s|op|t>; 0 for the zero operator.
int op_charge(const double *op, const Phys &p, const char *who) {
    const int d = p.d();
    int q = 0;
    bool seen = false;
    for (int a = 0; a < d; ++a)
        for (int b = 0; b < d; ++b)
            if (op[a * d + b] != 0.0) {
                const int c = p.q[a] - p.q[b];
                PD_REQUIRE(!seen || c == q, PDMRG_EINVAL, std::string(who) + ": operator without a definite charge");
                q = c;
                seen = true;
            }
    return q;
}

void check_mpo(const pdmrg_mps *m, const pdmrg_mpo *mpo) {
    PD_REQUIRE(mpo->N == m->N, PDMRG_ESHAPE, "sweep: MPO and MPS lengths differ");
    PD_REQUIRE(mpo->W[0].Dl == 1 && mpo->W[m->N - 1].Dr == 1, PDMRG_ESHAPE, "sweep: MPO boundary channels");
    PD_REQUIRE(mpo->d == m->p.d(), PDMRG_ESHAPE, "sweep: MPO local dimension differs from the MPS");
}

}  // namespace

#define API_TRY try {
#define API_CATCH                                   \
    }                                               \
    catch (const Error &e) {                        \
        set_last_error(e.what());                   \
        return e.code;                              \
    }                                               \
    catch (const std::exception &e) {               \
        set_last_error(e.what());                   \
        return PDMRG_EINVAL;                        \
    }                                               \
    return PDMRG_OK;

extern "C" {

int mps_alloc(pdmrg_ctx *ctx, int nsites, const pdmrg_phys *phys, int32_t q_target, const pdmrg_bond *bonds,
              pdmrg_mps **out) {
    API_TRY
    PD_REQUIRE(ctx && phys && bonds && out && nsites >= 2, PDMRG_EINVAL, "mps_alloc: bad arguments");
    auto m = std::make_unique<pdmrg_mps>();
    m->N = nsites;
    m->q_target = q_target;
    m->p = Phys::from(phys);
    for (int b = 0; b <= nsites; ++b) m->bonds.push_back(Bond::from(&bonds[b]));
    PD_REQUIRE(m->bonds[0].q == std::vector<int>{0} && m->bonds[0].dim == std::vector<int>{1}, PDMRG_ESHAPE,
               "mps_alloc: bond 0 must be {q=0, dim=1}");
    PD_REQUIRE(m->bonds[nsites].q == std::vector<int>{q_target} && m->bonds[nsites].dim == std::vector<int>{1},
               PDMRG_ESHAPE, "mps_alloc: last bond must be {q=target, dim=1}");
    m->sites.resize(nsites);
    m->V.resize(nsites + 1);
    m->Vd.resize(nsites + 1);
    m->hasV.assign(nsites + 1, 0);
    for (int i = 0; i < nsites; ++i) {
        const int64_t n = site_layout(m->bonds[i], m->bonds[i + 1], m->p).size;
        PD_REQUIRE(n > 0, PDMRG_ESHAPE, "mps_alloc: site " + std::to_string(i) + " has no allowed block");
        m->sites[i].alloc(n * sizeof(double));
        HIP_OK(hipMemsetAsync(m->sites[i].ptr, 0, n * sizeof(double), ctx->stream));
    }
    HIP_OK(hipStreamSynchronize(ctx->stream));
    *out = m.release();
    API_CATCH
}

int mps_set_site(pdmrg_mps *m, int site, const double *host_data, int64_t n) {
    API_TRY
    PD_REQUIRE(m && host_data && site >= 0 && site < m->N, PDMRG_EINVAL, "mps_set_site: bad arguments");
    const int64_t need = site_layout(m->bonds[site], m->bonds[site + 1], m->p).size;
    PD_REQUIRE(n == need, PDMRG_ESHAPE, "mps_set_site: expected " + std::to_string(need) + " elements");
    HIP_OK(hipMemcpy(m->sites[site].ptr, host_data, n * sizeof(double), hipMemcpyHostToDevice));
    m->ready = false;
    m->split = false;
    m->icanon = false;
    m->clear_v();
    API_CATCH
}

int mps_bond(const pdmrg_mps *m, int b, int32_t *nsec, int32_t *q, int32_t *dim, int32_t cap) {
    API_TRY
    PD_REQUIRE(m && b >= 0 && b <= m->N, PDMRG_EINVAL, "mps_bond: bad bond");
    const Bond &B = m->bonds[b];
    if (nsec) *nsec = B.nsec();
    if (q || dim) {
        PD_REQUIRE(cap >= B.nsec(), PDMRG_EINVAL, "mps_bond: capacity too small");
        for (int k = 0; k < B.nsec(); ++k) {
            if (q) q[k] = B.q[k];
            if (dim) dim[k] = B.dim[k];
        }
    }
    API_CATCH
}

int mps_get_site(pdmrg_mps *m, int site, double *host_data, int64_t cap) {
    API_TRY
    PD_REQUIRE(m && host_data && site >= 0 && site < m->N, PDMRG_EINVAL, "mps_get_site: bad arguments");
    const int64_t n = site_layout(m->bonds[site], m->bonds[site + 1], m->p).size;
    PD_REQUIRE(cap >= n, PDMRG_EINVAL, "mps_get_site: capacity too small");
    HIP_OK(hipMemcpy(host_data, m->sites[site].ptr, n * sizeof(double), hipMemcpyDeviceToHost));
    API_CATCH
}

int sweep(pdmrg_ctx *ctx, pdmrg_mps *m, const pdmrg_mpo *mpo, const pdmrg_sweep_params *p, pdmrg_sweep_report *rep) {
    API_TRY
    PD_REQUIRE(ctx && m && mpo && p, PDMRG_EINVAL, "sweep: null argument");
    check_mpo(m, mpo);
    PD_REQUIRE(p->max_m >= 1 && p->n_regions >= 1 && p->concurrent >= 0 && p->concurrent <= 2, PDMRG_EINVAL,
               "sweep: bad parameters");
    const auto t0 = std::chrono::steady_clock::now();
    Driver dr{ctx, m, mpo};
    dr.stride = ctx->env_stride;
    dr.prm = *p;
    if (m->icanon) dr.unsplit();   // fold V back before re-canonicalising
    if (!m->ready) dr.init();
    if (p->n_regions != m->n_regions || m->regions.empty()) {
        PD_REQUIRE(!m->split, PDMRG_EINVAL, "sweep: the region count cannot change after the split");
        const int size = m->N / p->n_regions;
        PD_REQUIRE(size >= 2 && size * p->n_regions == m->N, PDMRG_EINVAL,
                   "sweep: regions must hold >= 2 sites and tile the chain");
        m->n_regions = p->n_regions;
        m->regions.clear();
        for (int r = 0; r < p->n_regions; ++r) m->regions.push_back({r * size, (r + 1) * size - 1});
    }
    if (m->n_regions > 1 && !m->split) dr.split_regions();
    dr.parallel_sweep();
    const double E = dr.energy();
    if (rep) {
        *rep = dr.rep;
        rep->energy = E;
        rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        rep->seconds_heff = dr.t_heff;
        rep->seconds_svd = dr.t_svd;
        rep->seconds_env = dr.t_env;
    }
    API_CATCH
}

int mps_energy(pdmrg_ctx *ctx, pdmrg_mps *m, const pdmrg_mpo *mpo, double *energy) {
    API_TRY
    PD_REQUIRE(ctx && m && mpo && energy, PDMRG_EINVAL, "mps_energy: null argument");
    check_mpo(m, mpo);
    Driver dr{ctx, m, mpo};
    dr.stride = ctx->env_stride;
    *energy = dr.energy();
    API_CATCH
}

int grad_mpo(pdmrg_ctx *ctx, pdmrg_mps *m, const pdmrg_mpo *mpo, double *G_dev, int64_t n_G, double *energy) {
    API_TRY
    PD_REQUIRE(ctx && m && mpo && G_dev, PDMRG_EINVAL, "grad_mpo: null argument");
    check_mpo(m, mpo);
    std::vector<int64_t> goff(m->N + 1, 0);
    for (int i = 0; i < m->N; ++i) {
        const MpoSite &w = mpo->W[i];
        goff[i + 1] = goff[i] + (int64_t)w.Dl * w.d * w.d * w.Dr;
    }
    PD_REQUIRE(n_G == goff[m->N], PDMRG_ESHAPE, "grad_mpo: expected " + std::to_string(goff[m->N]) + " elements");
    Driver dr{ctx, m, mpo};
    dr.stride = ctx->env_stride;
    dr.prm.eps = 1e-4;
    if (energy) *energy = dr.energy();
    dr.gradients(G_dev, goff);
    API_CATCH
}

int grad_couplings(pdmrg_ctx *ctx, pdmrg_mps *m, const pdmrg_mpo *mpo, double *dE, int32_t ncouplings,
                   double *energy) {
    API_TRY
    PD_REQUIRE(ctx && m && mpo && dE && ncouplings >= 1, PDMRG_EINVAL, "grad_couplings: bad arguments");
    check_mpo(m, mpo);
    PD_REQUIRE((int)mpo->dW.size() == ncouplings, PDMRG_EINVAL,
               "grad_couplings: the MPO carries " + std::to_string(mpo->dW.size()) +
                   " coupling derivative tables (mpo_build MPOs only)");
    std::vector<int64_t> goff(m->N + 1, 0);
    for (int i = 0; i < m->N; ++i) {
        const MpoSite &w = mpo->W[i];
        goff[i + 1] = goff[i] + (int64_t)w.Dl * w.d * w.d * w.Dr;
    }
    const int64_t nG = goff[m->N];
    for (int k = 0; k < ncouplings; ++k)
        PD_REQUIRE((int64_t)mpo->dW[k].size() == nG, PDMRG_EINVAL,
                   "grad_couplings: the MPO's structure depends on coupling " + std::to_string(k));
    hipStream_t s = ctx->stream;
    DevBuf G((size_t)nG * sizeof(double));
    Driver dr{ctx, m, mpo};
    dr.stride = ctx->env_stride;
    dr.prm.eps = 1e-4;
    if (energy) *energy = dr.energy();
    dr.gradients(G.as<double>(), goff);
    // dE/dtheta_k = sum_i <G_i, dW_i/dtheta_k>: fixed-order tiled dot products
    std::vector<double> dWall;
    dWall.reserve((size_t)ncouplings * nG);
    for (int k = 0; k < ncouplings; ++k) dWall.insert(dWall.end(), mpo->dW[k].begin(), mpo->dW[k].end());
    std::vector<DotTask> tasks;
    std::vector<DotTile> tiles;
    std::vector<int32_t> t0, g_of;
    for (int k = 0; k < ncouplings; ++k) {
        tasks.push_back(DotTask{0, (int64_t)k * nG, (int32_t)nG, k});
        t0.push_back((int32_t)tiles.size());
        g_of.push_back(k);
        for (int64_t c = 0; c * kDotChunk < nG; ++c) tiles.push_back(DotTile{k, (int32_t)c});
    }
    t0.push_back((int32_t)tiles.size());
    PD_REQUIRE(nG < (int64_t(1) << 31), PDMRG_EINVAL, "grad_couplings: gradient too large");
    DevBuf d_dw, d_tasks, d_tiles, d_t0, d_g, partial, out;
    upload(d_dw, dWall, s);
    upload(d_tasks, tasks, s);
    upload(d_tiles, tiles, s);
    upload(d_t0, t0, s);
    upload(d_g, g_of, s);
    partial.ensure(std::max<size_t>(tiles.size(), 1) * sizeof(double));
    out.ensure((size_t)ncouplings * sizeof(double));
    Slots sl{};
    sl.p[0] = G.ptr;
    sl.p[1] = d_dw.ptr;
    launch_dot_partials(sl, 0, 1, d_tasks.as<DotTask>(), d_tiles.as<DotTile>(), (int)tiles.size(), partial.as<double>(), s);
    launch_dot_reduce(partial.as<double>(), d_t0.as<int32_t>(), d_g.as<int32_t>(), ncouplings, out.as<double>(), s);
    HIP_OK(hipMemcpyAsync(dE, out.ptr, (size_t)ncouplings * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    API_CATCH
}

int mps_inverse_canonical(pdmrg_ctx *ctx, pdmrg_mps *m, double cutoff, double eps, int32_t *n_floored) {
    API_TRY
    PD_REQUIRE(ctx && m, PDMRG_EINVAL, "mps_inverse_canonical: null argument");
    PD_REQUIRE(cutoff >= 0.0 && cutoff < 1.0 && eps >= 0.0 && eps < 1.0, PDMRG_EINVAL,
               "mps_inverse_canonical: cutoff and eps must lie in [0, 1)");
    Driver dr{ctx, m, nullptr};
    dr.prm.eps = eps;
    const int nfl = dr.inverse_canonical(cutoff);
    if (n_floored) *n_floored = nfl;
    API_CATCH
}

int mps_get_v(const pdmrg_mps *m, int bond, double *V, int64_t cap) {
    API_TRY
    PD_REQUIRE(m && V && bond >= 0 && bond <= m->N, PDMRG_EINVAL, "mps_get_v: bad arguments");
    PD_REQUIRE(m->hasV[bond] && m->split, PDMRG_EINVAL, "mps_get_v: no V on this bond");
    const std::vector<double> &v = m->V[bond];
    PD_REQUIRE(cap >= (int64_t)v.size(), PDMRG_EINVAL, "mps_get_v: capacity too small");
    std::copy(v.begin(), v.end(), V);
    API_CATCH
}

int mps_expect_site(pdmrg_ctx *ctx, pdmrg_mps *m, const double *op, double *out) {
    API_TRY
    PD_REQUIRE(ctx && m && op && out, PDMRG_EINVAL, "mps_expect_site: null argument");
    PD_REQUIRE(m->icanon, PDMRG_EINVAL, "mps_expect_site: the MPS is not in the inverse canonical gauge");
    const int d = m->p.d();
    Driver dr{ctx, m, nullptr};
    dr.expect_site(std::vector<double>(op, op + (size_t)d * d), out);
    API_CATCH
}

int mps_expect_pairs(pdmrg_ctx *ctx, pdmrg_mps *m, int nterms, const double *coef, const double *opA,
                     const double *opB, int npairs, const int32_t *site_i, const int32_t *site_k, int concurrent,
                     double *out) {
    API_TRY
    PD_REQUIRE(ctx && m && coef && opA && opB && out && nterms >= 1 && npairs >= 0 && (npairs == 0 || (site_i && site_k)),
               PDMRG_EINVAL, "mps_expect_pairs: bad arguments");
    PD_REQUIRE(m->icanon, PDMRG_EINVAL, "mps_expect_pairs: the MPS is not in the inverse canonical gauge");
    for (int p = 0; p < npairs; ++p)
        PD_REQUIRE(site_i[p] >= 0 && site_i[p] < site_k[p] && site_k[p] < m->N, PDMRG_EINVAL,
                   "mps_expect_pairs: each pair needs 0 <= i < k < N");
    const int d = m->p.d(), T = nterms;
    MpoSite Wi, Wm, Wk;
    Wi.Dl = 1, Wi.Dr = T, Wi.d = d;
    Wm.Dl = T, Wm.Dr = T, Wm.d = d;
    Wk.Dl = T, Wk.Dr = 1, Wk.d = d;
    Wi.W.assign((size_t)d * d * T, 0.0);
    Wm.W.assign((size_t)T * d * d * T, 0.0);
    Wk.W.assign((size_t)T * d * d, 0.0);
    std::vector<int> deltas(T);
    for (int t = 0; t < T; ++t) {
        const double *A = opA + (size_t)t * d * d, *B = opB + (size_t)t * d * d;
        deltas[t] = op_charge(A, m->p, "mps_expect_pairs");
        const int qb = op_charge(B, m->p, "mps_expect_pairs");
        bool bz = true;
        for (int e = 0; e < d * d; ++e) bz = bz && B[e] == 0.0;
        PD_REQUIRE(bz || qb == -deltas[t], PDMRG_EINVAL, "mps_expect_pairs: the charges of A_t and B_t must cancel");
        for (int a = 0; a < d; ++a)
            for (int b = 0; b < d; ++b) {
                Wi.W[((size_t)a * d + b) * T + t] = A[a * d + b];
                Wk.W[(((size_t)t * d + a) * d + b)] = coef[t] * B[a * d + b];
            }
        for (int a = 0; a < d; ++a) Wm.W[(((size_t)t * d + a) * d + a) * T + t] = 1.0;
    }
    Wi.dl = {0};
    Wi.dr = deltas;
    Wm.dl = deltas;
    Wm.dr = deltas;
    Wk.dl = deltas;
    Wk.dr = {0};
    Driver dr{ctx, m, nullptr};
    dr.prm.concurrent = concurrent ? 1 : 0;
    const int njobs = std::min(npairs, 8);
    std::vector<std::function<void(Driver &)>> jobs;
    for (int q = 0; q < njobs; ++q)
        jobs.push_back([=, &Wi, &Wm, &Wk](Driver &d) {
            for (int p = q; p < npairs; p += njobs) out[p] = d.correlator(site_i[p], site_k[p], Wi, Wm, Wk);
        });
    dr.run_jobs(jobs);
    API_CATCH
}

int mps_order_parameter(pdmrg_ctx *ctx, pdmrg_mps *m, int kind, int Lx, int Ly, double *value) {
    API_TRY
    PD_REQUIRE(ctx && m && value, PDMRG_EINVAL, "mps_order_parameter: null argument");
    PD_REQUIRE(m->icanon, PDMRG_EINVAL, "mps_order_parameter: the MPS is not in the inverse canonical gauge");
    PD_REQUIRE(Lx >= 1 && Ly >= 1 && Lx * Ly == m->N, PDMRG_EINVAL, "mps_order_parameter: Lx * Ly must equal N");
    PD_REQUIRE(m->p.d() == 2, PDMRG_EINVAL, "mps_order_parameter: spin-1/2 sites only");
    const double sz[4] = {0.5 * m->p.q[0], 0.0, 0.0, 0.5 * m->p.q[1]};
    // |up><down| and its transpose, up = the larger charge
    const int up = m->p.q[1] > m->p.q[0] ? 1 : 0, dn = 1 - up;
    double sp[4] = {0, 0, 0, 0}, sm[4] = {0, 0, 0, 0};
    sp[up * 2 + dn] = 1.0;
    sm[dn * 2 + up] = 1.0;
    Driver dr{ctx, m, nullptr};
    if (kind == 0) {
        // columnar dimer order D_x of the centre column x = Lx/2 - 1 (0-based)
        PD_REQUIRE(Lx >= 4, PDMRG_EINVAL, "mps_order_parameter: D_x needs Lx >= 4");
        const int xc = Lx / 2 - 1;
        std::vector<int32_t> si, sk;
        for (int o = -1; o <= 1; ++o)
            for (int y = 0; y < Ly; ++y) {
                const int a = lattice_snake(xc + o, y, Ly), b = lattice_snake(xc + o + 1, y, Ly);
                si.push_back(std::min(a, b));
                sk.push_back(std::max(a, b));
            }
        double A[12], B[12];
        const double coef[3] = {1.0, 0.5, 0.5};
        for (int e = 0; e < 4; ++e) {
            A[e] = sz[e], B[e] = sz[e];
            A[4 + e] = sp[e], B[4 + e] = sm[e];
            A[8 + e] = sm[e], B[8 + e] = sp[e];
        }
        std::vector<double> v(si.size());
        const int rc = mps_expect_pairs(ctx, m, 3, coef, A, B, (int)si.size(), si.data(), sk.data(), 0, v.data());
        if (rc != PDMRG_OK) return rc;
        double acc = 0.0;
        for (int y = 0; y < Ly; ++y) acc += v[Ly + y] - 0.5 * v[y] - 0.5 * v[2 * Ly + y];
        *value = acc / Ly;
    } else if (kind == 1) {
        // sublattice magnetisation M_z of the centre column x = (Lx - 1)/2 on
        // the pinned sublattice (x - y) mod 3 = 0
        PD_REQUIRE(Ly % 3 == 0, PDMRG_EINVAL, "mps_order_parameter: M_z needs Ly % 3 == 0");
        const int xc = (Lx - 1) / 2;
        std::vector<double> all(m->N);
        dr.expect_site(std::vector<double>(sz, sz + 4), all.data());
        double acc = 0.0;
        int n = 0;
        for (int y = 0; y < Ly; ++y)
            if (tri_sublattice(xc, y) == 0) {
                acc += all[lattice_snake(xc, y, Ly)];
                ++n;
            }
        *value = acc / n;
    } else {
        throw Error(PDMRG_EINVAL, "mps_order_parameter: kind must be 0 (D_x) or 1 (M_z)");
    }
    API_CATCH
}

int mps_copy(pdmrg_ctx *ctx, const pdmrg_mps *src, pdmrg_mps **out) {
    API_TRY
    PD_REQUIRE(ctx && src && out, PDMRG_EINVAL, "mps_copy: null argument");
    auto m = std::make_unique<pdmrg_mps>();
    m->N = src->N;
    m->q_target = src->q_target;
    m->p = src->p;
    m->bonds = src->bonds;
    m->V = src->V;
    m->hasV = src->hasV;
    m->ready = src->ready;
    m->n_regions = src->n_regions;
    m->split = src->split;
    m->icanon = src->icanon;
    m->regions = src->regions;
    auto dup = [&](const DevBuf &b) {
        DevBuf d;
        if (b.ptr) {
            d.alloc(b.bytes);
            HIP_OK(hipMemcpyAsync(d.ptr, b.ptr, b.bytes, hipMemcpyDeviceToDevice, ctx->stream));
        }
        return d;
    };
    for (const auto &b : src->sites) m->sites.push_back(dup(b));
    for (const auto &b : src->L) m->L.push_back(dup(b));
    for (const auto &b : src->R) m->R.push_back(dup(b));
    for (const auto &b : src->Vd) m->Vd.push_back(dup(b));
    HIP_OK(hipStreamSynchronize(ctx->stream));
    *out = m.release();
    API_CATCH
}

void mps_free(pdmrg_mps *m) { delete m; }

}  // extern "C"
