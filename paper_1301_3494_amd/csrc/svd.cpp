// Truncated SVD of the two-site wavefunction (Eq. eqn:svd) with the accurate
// recursive SVD of the Appendix, on the device.
//
// Psi viewed as the (m d) x (d m) matrix is block-diagonal in the middle
// charge; each block M (rows (s1, a), columns (s2, b)) is gathered densely and
// decomposed M = U Lambda Vt by one-sided block Jacobi (svd.hip); at the top
// level, blocks of at least 64 rows are first ordered by row norm and QR
// factored, and the iteration runs on the triangular factor (qr_factor,
// qr_right_factor: about half the sweeps on graded blocks).  Appendix
// recursion: for the singular values of a block below eps * lambda_1 (indices
// p..k-1), X = Ut[p:] M Vt[p:]^T is formed with FP64 GEMMs and decomposed the
// same way (recursively), then Ut[p:] <- Ut~ Ut[p:], Vt[p:] <- Vt~ Vt[p:],
// lambda[p:] <- lambda~ and the block is re-sorted.  Truncation keeps the
// max_m largest values over all blocks (ties: larger value, smaller charge,
// smaller index), drops lambda < cutoff * lambda_max, renormalises.
#include "internal.hpp"
#include "svd.hpp"

#include <cmath>
#include <cstdio>
#include <numeric>
#include <tuple>

namespace pdmrg {

namespace {

constexpr int kJacBlock = 8;
constexpr int kMaxSweeps = 60;
constexpr int kMaxDepth = 8;
// Smallest matrix (rows of W) that takes the QR preconditioning by default:
// below it the factorisation's launches cost more than the sweeps it saves.
constexpr int kQrMinRows = 64;
// Relative size (to a block's largest singular value) below which singular
// values are rounding noise of the FP64 block: the Appendix recursion does not
// descend into a trailing set that lies wholly below it.
constexpr double kNoise = 64.0 * 2.220446049250313e-16;

struct Arena {
    std::shared_ptr<DevBuf> buf = std::make_shared<DevBuf>();
    size_t cap = 0, used = 0;
    void reserve(size_t ndoubles) {
        buf->ensure(std::max<size_t>(ndoubles, 32) * sizeof(double));
        cap = buf->bytes / sizeof(double);
        used = 0;
    }
    double *take(size_t n) {
        n = (n + 31) & ~size_t(31);
        PD_REQUIRE(used + n <= cap, PDMRG_ENOMEM, "svd: arena overflow");
        double *p = buf->as<double>() + used;
        used += n;
        return p;
    }
    double *base() const { return buf->as<double>(); }
};

struct Mat {
    const double *M;   // device, row-major, ld = nc
    int nr, nc;
};

struct SvdRes {
    double *Ut = nullptr, *Vt = nullptr;   // k x nr, k x nc (device)
    std::vector<double> lam;               // k, descending
    int k = 0, nr = 0, nc = 0;
};

size_t round32(size_t n) { return (n + 31) & ~size_t(31); }

void run_copies(const std::vector<CopyTask> &tasks, hipStream_t s) {
    if (tasks.empty()) return;
    DevBuf d;
    upload(d, tasks, s);
    int64_t mx = 0;
    for (auto &t : tasks) mx = std::max<int64_t>(mx, (int64_t)t.rows * t.cols);
    launch_copies(d.as<CopyTask>(), (int)tasks.size(), mx, s);
    HIP_OK(hipStreamSynchronize(s));   // d is freed on return
}

// Householder QR preconditioning of the Jacobi iteration (depth 0).  The rows
// of a matrix's W (nv x len) are put in order of decreasing norm (P), the
// len x nv matrix X = (P W)^T is factored X = Q R, and the Jacobi iteration
// runs on the rows of R: Z R = D with orthogonal rows, so
// P W = R^T Q^T = D^T (Z Q^T).  R of a graded matrix is graded and its rows
// are close to orthogonal, so the iteration needs about half the sweeps.
// The factors: rows of D (length nv, norms = singular values) taken back
// through P, and Y = Z Q^T = [Z, 0] H_{nv-1} ... H_0 (length len), formed by
// applying the reflectors to [Z, 0] panel by panel, last panel first.
struct QrState {
    std::vector<int> len, inv_off;   // per matrix: row length of W; offset of P^-1 in d_idx
    std::vector<int32_t> idx;        // P then P^-1 per preconditioned matrix
    DevBuf d_idx, d_items, d_panels, d_trail, d_back;
    std::vector<QrItem> qitems;
    std::vector<QrPanel> panels;
    std::vector<QrApply> trail, back;
    std::vector<int> panel_off, trail_off, back_off, panel_span;
    int max_nv = 0;
    int64_t max_elems = 0;
};

void qr_factor(const std::vector<Mat> &mats, std::vector<JacItem> &items, const std::vector<char> &pre,
               const std::vector<double *> &qa, const std::vector<double *> &qm, const std::vector<double *> &qt,
               QrState &qs, hipStream_t s) {
    const int nm = (int)items.size();
    qs.len.assign(nm, 0);
    qs.inv_off.assign(nm, -1);
    // row norms of W, on the host: the order P (decreasing norm, then index)
    std::vector<RowRef> refs;
    std::vector<int> first(nm, 0);
    for (int i = 0; i < nm; ++i) {
        qs.len[i] = std::max(mats[i].nr, mats[i].nc);
        first[i] = (int)refs.size();
        if (!pre[i]) continue;
        for (int r = 0; r < items[i].nv; ++r) refs.push_back(RowRef{qm[i] + (size_t)r * qs.len[i], qs.len[i], 0});
    }
    DevBuf d_refs, d_norm;
    upload(d_refs, refs, s);
    d_norm.ensure(std::max<size_t>(refs.size(), 1) * sizeof(double));
    launch_row_norms(d_refs.as<RowRef>(), (int)refs.size(), d_norm.as<double>(), s);
    std::vector<double> norms(refs.size());
    HIP_OK(hipMemcpyAsync(norms.data(), d_norm.ptr, refs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    std::vector<int> perm_off(nm, -1);
    for (int i = 0; i < nm; ++i) {
        if (!pre[i]) continue;
        const int nv = items[i].nv;
        std::vector<int> perm(nv);
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(),
                         [&](int a, int b) { return norms[first[i] + a] > norms[first[i] + b]; });
        perm_off[i] = (int)qs.idx.size();
        qs.idx.insert(qs.idx.end(), perm.begin(), perm.end());
        qs.inv_off[i] = (int)qs.idx.size();
        qs.idx.resize(qs.idx.size() + nv);
        for (int r = 0; r < nv; ++r) qs.idx[qs.inv_off[i] + perm[r]] = r;
    }
    upload(qs.d_idx, qs.idx, s);
    // A = P W
    std::vector<CopyTask> cp;
    int64_t mx = 0;
    for (int i = 0; i < nm; ++i) {
        if (!pre[i]) continue;
        CopyTask t{};
        t.src = qm[i];
        t.dst = qa[i];
        t.rows = items[i].nv;
        t.cols = t.sld = t.dld = qs.len[i];
        t.ridx = qs.d_idx.as<int32_t>() + perm_off[i];
        cp.push_back(t);
        mx = std::max<int64_t>(mx, (int64_t)items[i].nv * qs.len[i]);
    }
    DevBuf d_cp;
    upload(d_cp, cp, s);
    launch_copies(d_cp.as<CopyTask>(), (int)cp.size(), mx, s);
    // panel task lists: factor, trailing update (Q^T), and later Y (from the right)
    int npan = 0;
    for (int i = 0; i < nm; ++i)
        if (pre[i]) {
            npan = std::max(npan, (items[i].nv + kQrPanel - 1) / kQrPanel);
            qs.max_nv = std::max(qs.max_nv, items[i].nv);
            qs.max_elems = std::max<int64_t>(qs.max_elems, (int64_t)items[i].nv * qs.len[i]);
            qs.qitems.push_back(QrItem{qa[i], items[i].Z, items[i].W, qm[i], items[i].nv, qs.len[i]});
        }
    for (int pn = 0; pn < npan; ++pn) {
        const int j0 = pn * kQrPanel;
        qs.panel_off.push_back((int)qs.panels.size());
        qs.trail_off.push_back((int)qs.trail.size());
        qs.back_off.push_back((int)qs.back.size());
        int span = 0;
        for (int i = 0; i < nm; ++i) {
            const int nv = items[i].nv, len = qs.len[i];
            if (!pre[i] || nv <= j0) continue;
            const int nb = std::min(kQrPanel, nv - j0);
            double *T = qt[i] + (size_t)pn * kQrPanel * kQrPanel;
            qs.panels.push_back(QrPanel{qa[i], T, nv, len, j0, 0});
            span = std::max(span, len - j0);
            for (int g0 = j0 + nb; g0 < nv; g0 += kQrPanel)
                qs.trail.push_back(QrApply{qa[i] + (size_t)j0 * len, T, qa[i] + (size_t)g0 * len, nb,
                                           std::min(kQrPanel, nv - g0), len, j0, 1, 0});
            for (int g0 = 0; g0 < nv; g0 += kQrPanel)
                qs.back.push_back(QrApply{qa[i] + (size_t)j0 * len, T, qm[i] + (size_t)g0 * len, nb,
                                          std::min(kQrPanel, nv - g0), len, j0, 0, 0});
        }
        qs.panel_span.push_back(span);
    }
    qs.panel_off.push_back((int)qs.panels.size());
    qs.trail_off.push_back((int)qs.trail.size());
    qs.back_off.push_back((int)qs.back.size());
    upload(qs.d_items, qs.qitems, s);
    upload(qs.d_panels, qs.panels, s);
    upload(qs.d_trail, qs.trail, s);
    upload(qs.d_back, qs.back, s);
    for (int pn = 0; pn < npan; ++pn) {
        launch_qr_panels(qs.d_panels.as<QrPanel>() + qs.panel_off[pn], qs.panel_off[pn + 1] - qs.panel_off[pn],
                         qs.panel_span[pn], s);
        launch_qr_apply(qs.d_trail.as<QrApply>() + qs.trail_off[pn], qs.trail_off[pn + 1] - qs.trail_off[pn], s);
    }
    // the Jacobi iteration's rows: R
    launch_qr_extract_r(qs.d_items.as<QrItem>(), (int)qs.qitems.size(), qs.max_nv, s);
    HIP_OK(hipStreamSynchronize(s));   // d_refs, d_norm, d_cp are freed on return
}

void qr_right_factor(QrState &qs, hipStream_t s) {
    launch_qr_embed_z(qs.d_items.as<QrItem>(), (int)qs.qitems.size(), qs.max_elems, s);
    for (int pn = (int)qs.panel_span.size() - 1; pn >= 0; --pn)
        launch_qr_apply(qs.d_back.as<QrApply>() + qs.back_off[pn], qs.back_off[pn + 1] - qs.back_off[pn], s);
}

// One-sided block Jacobi on every matrix; returns sorted factors in `arena`.
// floor (one per matrix, used from depth 1 on): values below it are rounding
// noise of the block at depth 0, where the recursion stops.  n_unconv is
// incremented by the number of blocks (at any depth) whose Jacobi iteration
// did not meet its tolerance within kMaxSweeps sweeps.
void svd_batch(pdmrg_ctx *ctx, const std::vector<Mat> &mats, std::vector<SvdRes> &out, double eps, int depth,
               std::vector<Arena> &keep, const std::vector<double> &floor, int &n_unconv) {
    hipStream_t s = ctx->stream;
    const int nm = (int)mats.size();
    out.assign(nm, SvdRes());
    if (nm == 0) return;
    // QR preconditioning (depth 0): which matrices take it
    std::vector<char> pre(nm, 0);
    bool any_pre = false;
    for (int i = 0; i < nm; ++i) {
        const int nv = std::min(mats[i].nr, mats[i].nc), len = std::max(mats[i].nr, mats[i].nc);
        pre[i] = depth == 0 && ctx->svd_precond > 0 && nv >= (ctx->svd_precond >= 2 ? 2 : kQrMinRows) &&
                 len <= kQrMaxLen;
        any_pre = any_pre || pre[i];
    }
    Arena ar;
    size_t need = 64;
    for (int i = 0; i < nm; ++i) {
        const Mat &m = mats[i];
        const size_t nv = std::min(m.nr, m.nc), len = std::max(m.nr, m.nc);
        need += round32(nv * len) + round32(nv * nv) + round32(nv * m.nr) + round32(nv * m.nc) + round32(nv) + 96;
        if (pre[i]) need += round32(nv * len) + round32(nv * nv) + round32((nv + kQrPanel - 1) / kQrPanel * 256) + 96;
    }
    ar.reserve(need);
    std::vector<JacItem> items(nm);
    std::vector<CopyTask> cp;
    // per preconditioned matrix: A (QR storage), the copy of M (later Y), R, T
    std::vector<double *> qa(nm, nullptr), qm(nm, nullptr), qt(nm, nullptr);
    for (int i = 0; i < nm; ++i) {
        const Mat &m = mats[i];
        const bool wide = m.nr <= m.nc;
        const int nv = std::min(m.nr, m.nc), len = std::max(m.nr, m.nc);
        // the Jacobi kernel addresses W and Z with 32-bit byte offsets
        PD_REQUIRE((int64_t)nv * len * 8 < (int64_t(1) << 31), PDMRG_EINVAL, "svd: block too large");
        items[i].nv = nv;
        items[i].len = pre[i] ? nv : len;
        // each matrix on its own tolerance, so a matrix's rotations do not
        // depend on which others share its launches
        items[i].tol = std::max(1e-14, 8.0 * 2.220446049250313e-16 * std::sqrt((double)items[i].len));
        double *wm = ar.take((size_t)nv * len);
        if (pre[i]) {
            qm[i] = wm;
            qa[i] = ar.take((size_t)nv * len);
            qt[i] = ar.take((size_t)(nv + kQrPanel - 1) / kQrPanel * 256);
            items[i].W = ar.take((size_t)nv * nv);   // rows of R
        } else {
            items[i].W = wm;
        }
        items[i].Z = ar.take((size_t)nv * nv);
        out[i].nr = m.nr;
        out[i].nc = m.nc;
        out[i].k = nv;
        out[i].Ut = ar.take((size_t)nv * m.nr);
        out[i].Vt = ar.take((size_t)nv * m.nc);
        CopyTask t{};
        t.src = m.M;
        t.dst = wm;
        t.rows = nv;
        t.cols = len;
        t.sld = m.nc;
        t.dld = len;
        t.trans = wide ? 0 : 1;   // tall: W = M^T
        cp.push_back(t);
    }
    run_copies(cp, s);
    QrState qs;
    if (any_pre) qr_factor(mats, items, pre, qa, qm, qt, qs, s);
    DevBuf d_items;
    upload(d_items, items, s);
    int max_nv = 0;
    for (auto &it : items) max_nv = std::max(max_nv, it.nv);
    launch_identity(d_items.as<JacItem>(), nm, max_nv, s);

    // circle schedule over blocks of 8 rows
    std::vector<int> nblk(nm);
    int rmax = 0;
    for (int i = 0; i < nm; ++i) {
        int nb = std::max(2, (items[i].nv + kJacBlock - 1) / kJacBlock);
        if (nb % 2) ++nb;
        nblk[i] = nb;
        rmax = std::max(rmax, nb - 1);
    }
    std::vector<std::vector<JacPair>> rounds(rmax);
    for (int i = 0; i < nm; ++i) {
        const int nb = nblk[i], real = (items[i].nv + kJacBlock - 1) / kJacBlock;
        for (int r = 0; r < nb - 1; ++r)
            for (int l = 0; l < nb / 2; ++l) {
                const int p = (l == 0) ? nb - 1 : (r + l) % (nb - 1);
                const int q = (r - l + (nb - 1)) % (nb - 1);
                if (p >= real && q >= real) continue;
                rounds[r].push_back(JacPair{i, std::min(p, q), std::max(p, q), 0});
            }
    }
    std::vector<JacPair> flat;
    std::vector<int> roff(rmax + 1, 0);
    for (int r = 0; r < rmax; ++r) {
        roff[r] = (int)flat.size();
        flat.insert(flat.end(), rounds[r].begin(), rounds[r].end());
    }
    roff[rmax] = (int)flat.size();
    DevBuf d_pairs, d_active, d_off;
    upload(d_pairs, flat, s);
    std::vector<int32_t> active(nm, 1);
    d_off.ensure(std::max(nm, 1) * sizeof(unsigned long long));

    int sweeps_done = 0, nrounds = 0;
    for (int sweep = 0; sweep < kMaxSweeps; ++sweep) {
        sweeps_done = sweep + 1;
        upload(d_active, active, s);
        launch_fill(d_off.as<double>(), 0.0, nm, s);
        // rounds past every active matrix's last hold only pairs of converged
        // matrices, which do nothing: not launched
        int ract = 0;
        for (int i = 0; i < nm; ++i)
            if (active[i]) ract = std::max(ract, nblk[i] - 1);
        nrounds += ract;
        for (int r = 0; r < ract; ++r)
            launch_jac_round(d_items.as<JacItem>(), d_pairs.as<JacPair>() + roff[r], roff[r + 1] - roff[r],
                             d_active.as<int32_t>(), d_off.as<unsigned long long>(), s);
        std::vector<double> off(nm);
        HIP_OK(hipMemcpyAsync(off.data(), d_off.ptr, nm * sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        bool any = false;
        for (int i = 0; i < nm; ++i) {
            if (active[i] && off[i] <= items[i].tol) active[i] = 0;
            any = any || active[i];
        }
        if (!any) break;
    }
    // blocks whose rows were not orthogonal to tol after kMaxSweeps sweeps:
    // still an exact rotation of the block (absolute accuracy), reported
    for (int i = 0; i < nm; ++i) n_unconv += active[i] ? 1 : 0;
    if (any_pre) qr_right_factor(qs, s);
    if (ctx->verbose >= 2) {
        int big = 0, npre = 0;
        for (int i = 0; i < nm; ++i) {
            big = std::max(big, items[i].nv);
            npre += pre[i] ? 1 : 0;
        }
        std::fprintf(stderr,
                     "pdmrg: svd level %d: %d blocks (%d preconditioned), largest %d rows, %d sweeps, %d rounds\n",
                     depth, nm, npre, big, sweeps_done, nrounds);
    }

    // singular values = row norms
    std::vector<RowRef> refs;
    std::vector<int> first(nm + 1, 0);
    for (int i = 0; i < nm; ++i) {
        first[i] = (int)refs.size();
        for (int r = 0; r < items[i].nv; ++r) refs.push_back(RowRef{items[i].W + (size_t)r * items[i].len, items[i].len, 0});
    }
    first[nm] = (int)refs.size();
    DevBuf d_refs, d_norm;
    upload(d_refs, refs, s);
    d_norm.ensure(std::max<size_t>(refs.size(), 1) * sizeof(double));
    launch_row_norms(d_refs.as<RowRef>(), (int)refs.size(), d_norm.as<double>(), s);
    std::vector<double> norms(refs.size());
    if (!refs.empty())
        HIP_OK(hipMemcpyAsync(norms.data(), d_norm.ptr, refs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));

    // sorted factors: wide Ut = Z rows, Vt = W rows / lambda; tall the reverse
    std::vector<double> scales;
    std::vector<CopyTask> gt;
    std::vector<std::tuple<const double *, double *, int, int>> rowjobs;   // src, dst, len, scale index
    std::vector<int> gidx;   // per row job: offset of its column gather map in qs.d_idx, or -1
    for (int i = 0; i < nm; ++i) {
        const int nv = items[i].nv;
        std::vector<int> perm(nv);
        std::iota(perm.begin(), perm.end(), 0);
        std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return norms[first[i] + a] > norms[first[i] + b]; });
        const bool wide = mats[i].nr <= mats[i].nc;
        out[i].lam.resize(nv);
        for (int j = 0; j < nv; ++j) {
            const double l = norms[first[i] + perm[j]];
            out[i].lam[j] = l;
            const double *wrow = items[i].W + (size_t)perm[j] * items[i].len;
            const double *zrow = items[i].Z + (size_t)perm[j] * nv;
            const double inv = l > 0.0 ? 1.0 / l : 0.0;
            if (pre[i]) {
                // X P = Q R with R = Z^T D: the D row (W side) scattered back
                // through the row order P, scaled by 1 / lambda, and Y = Z Q^T
                const int len = std::max(mats[i].nr, mats[i].nc);
                const double *yrow = qm[i] + (size_t)perm[j] * len;
                double *dside = wide ? out[i].Ut + (size_t)j * mats[i].nr : out[i].Vt + (size_t)j * mats[i].nc;
                double *yside = wide ? out[i].Vt + (size_t)j * mats[i].nc : out[i].Ut + (size_t)j * mats[i].nr;
                rowjobs.emplace_back(wrow, dside, nv, (int)scales.size());
                scales.push_back(inv);
                gidx.push_back(qs.inv_off[i]);
                rowjobs.emplace_back(yrow, yside, len, (int)scales.size());
                scales.push_back(1.0);
                gidx.push_back(-1);
            } else if (wide) {
                rowjobs.emplace_back(zrow, out[i].Ut + (size_t)j * mats[i].nr, nv, (int)scales.size());
                scales.push_back(1.0);
                rowjobs.emplace_back(wrow, out[i].Vt + (size_t)j * mats[i].nc, items[i].len, (int)scales.size());
                scales.push_back(inv);
            } else {
                rowjobs.emplace_back(wrow, out[i].Ut + (size_t)j * mats[i].nr, items[i].len, (int)scales.size());
                scales.push_back(inv);
                rowjobs.emplace_back(zrow, out[i].Vt + (size_t)j * mats[i].nc, nv, (int)scales.size());
                scales.push_back(1.0);
            }
            if (!pre[i]) {
                gidx.push_back(-1);
                gidx.push_back(-1);
            }
        }
    }
    DevBuf d_scales;
    upload(d_scales, scales, s);
    for (size_t r = 0; r < rowjobs.size(); ++r) {
        auto &[src, dst, len, si] = rowjobs[r];
        CopyTask t{};
        t.src = src;
        t.dst = dst;
        t.rows = 1;
        t.cols = len;
        t.sld = len;
        t.dld = len;
        t.rscale = d_scales.as<double>() + si;
        if (gidx[r] >= 0) t.cidx = qs.d_idx.as<int32_t>() + gidx[r];
        gt.push_back(t);
    }
    run_copies(gt, s);

    // Appendix recursion on the trailing singular values
    {
        std::vector<int> who, pstart;
        std::vector<double> subfloor;
        for (int i = 0; i < nm; ++i) {
            const auto &l = out[i].lam;
            if (l.empty() || !(l[0] > 0.0)) continue;
            int p = -1;
            for (int j = 0; j < (int)l.size(); ++j)
                if (l[j] < eps * l[0]) { p = j; break; }
            if (p < 0) continue;
            // trailing values all below the noise floor of the original block
            // (kNoise of its largest value) carry no information to recover
            const double fl = depth == 0 ? kNoise * l[0] : floor[i];
            if (!(l[p] >= fl)) continue;
            who.push_back(i);
            pstart.push_back(p);
            subfloor.push_back(fl);
        }
        if (!who.empty()) {
            PD_REQUIRE(depth < kMaxDepth, PDMRG_ENUMERIC,
                       "svd: Appendix recursion still finds values below eps after " + std::to_string(kMaxDepth) +
                           " levels");
            Arena sub;
            size_t need2 = 64;
            for (size_t w = 0; w < who.size(); ++w) {
                const SvdRes &o = out[who[w]];
                const size_t t = o.k - pstart[w];
                need2 += round32(t * o.nc) + round32(t * t) + round32(t * std::max(o.nr, o.nc)) + 64;
            }
            sub.reserve(need2);
            // slots: 0 current arena (Ut, Vt, M lives elsewhere -> slot 2), 1 sub arena
            GemmList gy, gx;
            gx.tb = true;
            std::vector<Mat> subs;
            std::vector<double *> Y(who.size()), X(who.size()), T(who.size());
            const double *Mbase = mats[0].M;
            for (const Mat &m : mats) Mbase = std::min(Mbase, m.M);
            for (size_t w = 0; w < who.size(); ++w) {
                const SvdRes &o = out[who[w]];
                const int p = pstart[w], t = o.k - p;
                Y[w] = sub.take((size_t)t * o.nc);
                X[w] = sub.take((size_t)t * t);
                T[w] = sub.take((size_t)t * std::max(o.nr, o.nc));
                // Y = Ut[p:] (t x nr) M (nr x nc)
                gy.add_item(1, Y[w] - sub.base(), t, o.nc, o.nc);
                gy.add_seg(0, (o.Ut + (size_t)p * o.nr) - ar.base(), o.nr, 2, mats[who[w]].M - Mbase, o.nc, o.nr);
                // X = Y Vt[p:]^T (t x t)
                gx.add_item(1, X[w] - sub.base(), t, t, t);
                gx.add_seg(1, Y[w] - sub.base(), o.nc, 0, (o.Vt + (size_t)p * o.nc) - ar.base(), o.nc, o.nc);
                subs.push_back(Mat{X[w], t, t});
            }
            Slots sl{};
            sl.p[0] = ar.base();
            sl.p[1] = sub.base();
            sl.p[2] = Mbase;
            gy.finish(s);
            gy.launch(GemmPrec::F64, true, sl, s);
            gx.finish(s);
            gx.launch(GemmPrec::F64, true, sl, s);
            HIP_OK(hipStreamSynchronize(s));
            std::vector<SvdRes> so;
            svd_batch(ctx, subs, so, eps, depth + 1, keep, subfloor, n_unconv);
            // Ut[p:] <- Ut~ Ut[p:] ; Vt[p:] <- Vt~ Vt[p:]  (via T, then copy back)
            const double *SB = so[0].Ut;
            for (auto &r : so) SB = std::min<const double *>(SB, std::min(r.Ut, r.Vt));
            std::vector<CopyTask> back;
            for (int pass = 0; pass < 2; ++pass) {
                GemmList gu;
                for (size_t w = 0; w < who.size(); ++w) {
                    SvdRes &o = out[who[w]];
                    const int p = pstart[w], t = o.k - p;
                    const int len = pass == 0 ? o.nr : o.nc;
                    double *base = pass == 0 ? o.Ut : o.Vt;
                    const double *small = pass == 0 ? so[w].Ut : so[w].Vt;
                    gu.add_item(1, T[w] - sub.base(), t, len, len);
                    gu.add_seg(3, small - SB, t, 0, (base + (size_t)p * len) - ar.base(), len, t);
                    CopyTask c{};
                    c.src = T[w];
                    c.dst = base + (size_t)p * len;
                    c.rows = t;
                    c.cols = len;
                    c.sld = len;
                    c.dld = len;
                    back.push_back(c);
                }
                Slots s2{};
                s2.p[0] = ar.base();
                s2.p[1] = sub.base();
                s2.p[3] = SB;
                gu.finish(s);
                gu.launch(GemmPrec::F64, true, s2, s);
                run_copies(back, s);
                back.clear();
            }
            // new trailing values; re-sort each block
            std::vector<CopyTask> perm_tasks, perm_back;
            for (size_t w = 0; w < who.size(); ++w) {
                SvdRes &o = out[who[w]];
                const int p = pstart[w];
                for (int j = p; j < o.k; ++j) o.lam[j] = so[w].lam[j - p];
                std::vector<int> perm(o.k);
                std::iota(perm.begin(), perm.end(), 0);
                std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return o.lam[a] > o.lam[b]; });
                bool same = true;
                for (int j = 0; j < o.k; ++j) same = same && perm[j] == j;
                if (same) continue;
                std::vector<double> nl(o.k);
                for (int j = 0; j < o.k; ++j) nl[j] = o.lam[perm[j]];
                o.lam = nl;
                // stage into T-sized scratch: reuse a fresh buffer
                auto tmp = std::make_shared<DevBuf>((size_t)o.k * (o.nr + o.nc) * sizeof(double));
                keep.push_back(Arena{tmp, 0, 0});
                double *tu = tmp->as<double>(), *tv = tu + (size_t)o.k * o.nr;
                for (int j = 0; j < o.k; ++j) {
                    perm_tasks.push_back(CopyTask{o.Ut + (size_t)perm[j] * o.nr, tu + (size_t)j * o.nr, nullptr, nullptr,
                                                  1, o.nr, o.nr, o.nr, 0, 0});
                    perm_tasks.push_back(CopyTask{o.Vt + (size_t)perm[j] * o.nc, tv + (size_t)j * o.nc, nullptr, nullptr,
                                                  1, o.nc, o.nc, o.nc, 0, 0});
                }
                perm_back.push_back(CopyTask{tu, o.Ut, nullptr, nullptr, o.k, o.nr, o.nr, o.nr, 0, 0});
                perm_back.push_back(CopyTask{tv, o.Vt, nullptr, nullptr, o.k, o.nc, o.nc, o.nc, 0, 0});
            }
            run_copies(perm_tasks, s);
            run_copies(perm_back, s);
            keep.push_back(sub);
        }
    }
    keep.push_back(ar);
}

}  // namespace

namespace {
// Middle-charge sector block of one problem: rows (s1, i), columns (s2, k),
// gathered densely at M.
struct Sec {
    int qm, nr = 0, nc = 0;
    std::vector<std::pair<int, int>> rows;   // (s1, i)
    std::vector<std::pair<int, int>> cols;   // (s2, k)
    const double *M = nullptr;
};

std::vector<Sec> middle_sectors(const Bond &bl, const Bond &br, const Phys &p) {
    const int d = p.d();
    std::vector<int> mids;
    for (int i = 0; i < bl.nsec(); ++i)
        for (int s1 = 0; s1 < d; ++s1) mids.push_back(bl.q[i] + p.q[s1]);
    std::sort(mids.begin(), mids.end());
    mids.erase(std::unique(mids.begin(), mids.end()), mids.end());
    std::vector<Sec> secs;
    for (int qm : mids) {
        Sec sc;
        sc.qm = qm;
        for (int s2 = 0; s2 < d; ++s2) {
            const int k = br.find(qm + p.q[s2]);
            if (k >= 0) { sc.cols.push_back({s2, k}); sc.nc += br.dim[k]; }
        }
        for (int s1 = 0; s1 < d; ++s1) {
            const int i = bl.find(qm - p.q[s1]);
            if (i >= 0 && sc.nc > 0) { sc.rows.push_back({s1, i}); sc.nr += bl.dim[i]; }
        }
        if (sc.nr > 0 && sc.nc > 0) secs.push_back(sc);
    }
    return secs;
}

// Global truncation of one problem from its blocks' factors, and its output
// tensors (Eq. eqn:svd; modes as in svd_truncate).
void finish_problem(pdmrg_ctx *ctx, const SvdProblem &pb, const std::vector<Sec> &secs, const SvdRes *res,
                    SvdOut &out) {
    hipStream_t s = ctx->stream;
    const Bond &bl = *pb.bl, &br = *pb.br;
    const Phys &p = *pb.p;
    const int d = p.d();
    const int max_m = pb.max_m, mode = pb.mode;
    const double cutoff = pb.cutoff;
    // global truncation
    struct Cand { double l; int q, idx, sec; };
    std::vector<Cand> cand;
    double total = 0.0;
    for (size_t k = 0; k < secs.size(); ++k)
        for (int j = 0; j < res[k].k; ++j) {
            cand.push_back(Cand{res[k].lam[j], secs[k].qm, j, (int)k});
            total += res[k].lam[j] * res[k].lam[j];
        }
    std::sort(cand.begin(), cand.end(), [](const Cand &a, const Cand &b) {
        if (a.l != b.l) return a.l > b.l;
        if (a.q != b.q) return a.q < b.q;
        return a.idx < b.idx;
    });
    PD_REQUIRE(!cand.empty() && cand[0].l > 0.0, PDMRG_ENUMERIC, "svd_truncate: zero wavefunction");
    const double lmax = cand[0].l;
    std::vector<int> kept(secs.size(), 0);
    for (size_t c = 0; c < cand.size() && (int)c < max_m; ++c)
        if (cand[c].l >= cutoff * lmax && cand[c].l > 0.0) kept[cand[c].sec] += 1;
    double kept_w = 0.0;
    std::vector<int> nq, nd;
    std::vector<int> secidx;
    for (size_t k = 0; k < secs.size(); ++k) {
        if (kept[k] == 0) continue;
        for (int j = 0; j < kept[k]; ++j) kept_w += res[k].lam[j] * res[k].lam[j];
        nq.push_back(secs[k].qm);
        nd.push_back(kept[k]);
        secidx.push_back((int)k);
    }
    const double scale = 1.0 / std::sqrt(kept_w);
    out.bl = bl;
    out.br = br;
    out.p = p;
    out.mode = mode;
    out.bnew = Bond(nq, nd);
    out.discarded = std::max(0.0, 1.0 - kept_w / total);
    out.lam.clear();
    out.V.clear();
    out.n_floored = 0;
    for (size_t t = 0; t < secidx.size(); ++t)
        for (int j = 0; j < nd[t]; ++j) out.lam.push_back(res[secidx[t]].lam[j] * scale);
    const double lm = *std::max_element(out.lam.begin(), out.lam.end());
    for (double l : out.lam) {
        const double fl = std::max(l, 1e-12 * lm);
        if (l < 1e-12 * lm) out.n_floored += 1;
        out.V.push_back(1.0 / fl);
    }
    DevBuf d_lam;
    upload(d_lam, out.lam, s);
    const SiteLayout SA = site_layout(bl, out.bnew, p), SB = site_layout(out.bnew, br, p);
    out.A.ensure(std::max<int64_t>(SA.size, 1) * sizeof(double));
    out.B.ensure(std::max<int64_t>(SB.size, 1) * sizeof(double));
    out.left.ensure(std::max<int64_t>(SA.size, 1) * sizeof(double));
    out.right.ensure(std::max<int64_t>(SB.size, 1) * sizeof(double));
    std::vector<CopyTask> ct;
    for (size_t t = 0; t < secidx.size(); ++t) {
        const Sec &sc = secs[secidx[t]];
        const SvdRes &r = res[secidx[t]];
        const int kq = nd[t];
        const double *lam_q = d_lam.as<double>() + out.bnew.off[t];
        int r0 = 0;
        for (auto [s1, i] : sc.rows) {
            const int co = SA.colo[(size_t)i * d + s1];
            PD_REQUIRE(co >= 0, PDMRG_ESHAPE, "svd_truncate: output layout mismatch");
            for (int pass = 0; pass < 2; ++pass) {
                CopyTask c{};
                c.src = r.Ut + r0;           // element (a, alpha) = Ut[alpha][r0 + a]
                c.sld = r.nr;
                c.trans = 1;
                c.dst = (pass == 0 ? out.A.as<double>() : out.left.as<double>()) + SA.base[i] + co;
                c.dld = SA.cols[i];
                c.rows = bl.dim[i];
                c.cols = kq;
                c.cscale = pass == 0 ? nullptr : lam_q;
                ct.push_back(c);
            }
            r0 += bl.dim[i];
        }
        PD_REQUIRE(SB.cols[t] == sc.nc, PDMRG_ESHAPE, "svd_truncate: right layout mismatch");
        for (int pass = 0; pass < 2; ++pass) {
            CopyTask c{};
            c.src = r.Vt;
            c.sld = r.nc;
            c.dst = (pass == 0 ? out.B.as<double>() : out.right.as<double>()) + SB.base[t];
            c.dld = SB.cols[t];
            c.rows = kq;
            c.cols = sc.nc;
            c.rscale = pass == 0 ? nullptr : lam_q;
            ct.push_back(c);
        }
    }
    run_copies(ct, s);
}

}  // namespace

void svd_truncate_multi(pdmrg_ctx *ctx, const std::vector<SvdProblem> &probs, double eps,
                        std::vector<SvdOut> &outs) {
    hipStream_t s = ctx->stream;
    const int np = (int)probs.size();
    outs.clear();
    outs.resize(np);
    if (np == 0) return;
    std::vector<std::vector<Sec>> secs(np);
    size_t need = 64;
    for (int t = 0; t < np; ++t) {
        const SvdProblem &pb = probs[t];
        PD_REQUIRE(pb.mode >= 0 && pb.mode <= 2, PDMRG_EINVAL, "svd_truncate: bad mode");
        PD_REQUIRE(pb.max_m >= 1, PDMRG_EINVAL, "svd_truncate: max_m must be >= 1");
        secs[t] = middle_sectors(*pb.bl, *pb.br, *pb.p);
        for (auto &sc : secs[t]) need += round32((size_t)sc.nr * sc.nc);
    }
    ctx->ws_svd.ensure(need * sizeof(double));
    double *mbase = ctx->ws_svd.as<double>();
    size_t off = 0;
    std::vector<CopyTask> gather;
    std::vector<Mat> mats;
    std::vector<int> first(np + 1, 0);
    for (int t = 0; t < np; ++t) {
        const SvdProblem &pb = probs[t];
        const Bond &bl = *pb.bl;
        const int d = pb.p->d();
        const SiteLayout X = two_site_layout(*pb.bl, *pb.br, *pb.p);
        first[t] = (int)mats.size();
        for (auto &sc : secs[t]) {
            double *M = mbase + off;
            off += round32((size_t)sc.nr * sc.nc);
            sc.M = M;
            int r0 = 0;
            for (auto [s1, i] : sc.rows) {
                int col0 = -1;
                for (auto [s2, k] : sc.cols) {
                    const int co = X.colo[(size_t)i * d * d + s1 * d + s2];
                    PD_REQUIRE(co >= 0, PDMRG_ESHAPE, "svd_truncate: missing block");
                    if (col0 < 0) col0 = co;
                }
                CopyTask c{};
                c.src = pb.psi + X.base[i] + col0;
                c.dst = M + (size_t)r0 * sc.nc;
                c.rows = bl.dim[i];
                c.cols = sc.nc;
                c.sld = X.cols[i];
                c.dld = sc.nc;
                gather.push_back(c);
                r0 += bl.dim[i];
            }
            mats.push_back(Mat{M, sc.nr, sc.nc});
        }
    }
    first[np] = (int)mats.size();
    run_copies(gather, s);
    // every block of every problem in one batch: one launch per Jacobi round
    // for all of them (each block keeps its own tolerance, so its factors are
    // those of a batch of its own)
    std::vector<SvdRes> res;
    std::vector<Arena> keep;
    int n_unconv = 0;
    svd_batch(ctx, mats, res, eps, 0, keep, {}, n_unconv);
    for (int t = 0; t < np; ++t) {
        finish_problem(ctx, probs[t], secs[t], res.data() + first[t], outs[t]);
        outs[t].n_unconverged = t == 0 ? n_unconv : 0;   // the batch's count, reported once
    }
}

void svd_truncate_run(pdmrg_ctx *ctx, const Bond &bl, const Bond &br, const Phys &p, const double *psi, int max_m,
                      double cutoff, double eps, int mode, SvdOut &out) {
    std::vector<SvdOut> outs;
    svd_truncate_multi(ctx, {SvdProblem{&bl, &br, &p, psi, max_m, cutoff, mode}}, eps, outs);
    out = std::move(outs[0]);
}

}  // namespace pdmrg
