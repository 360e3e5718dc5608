// Two-site effective Hamiltonian operator (Sec. II): plan + environments in
// the compute precision + intermediates.
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <sstream>

#include "internal.hpp"

namespace pdmrg {

namespace {
std::mutex g_tune_mu;
struct Tuned {
    int shape1 = -1, shape3 = -1, parts3 = 0;
};
std::map<std::string, Tuned> &tune_cache() {
    static auto *m = new std::map<std::string, Tuned>();
    return *m;
}

std::string tune_key(int device, int prec, const Bond &bl, const Bond &br, const MpoSite &W1, const MpoSite &W2) {
    std::ostringstream o;
    o << device << '|' << prec << '|';
    for (int k = 0; k < bl.nsec(); ++k) o << bl.q[k] << ':' << bl.dim[k] << ',';
    o << '|';
    for (int k = 0; k < br.nsec(); ++k) o << br.q[k] << ':' << br.dim[k] << ',';
    o << '|' << W1.Dl << ',' << W1.Dr << ',' << W2.Dr << ',' << W1.d;
    for (int w : W1.dl) o << ',' << w;
    for (int w : W2.dr) o << ',' << w;
    return o.str();
}

// Average time (ms) of `reps` runs of fn on stream s after one warm-up run.
template <class F>
double time_ms(hipStream_t s, int reps, F &&fn) {
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    fn();
    HIP_OK(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) fn();
    HIP_OK(hipEventRecord(e1, s));
    HIP_OK(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_OK(hipEventElapsedTime(&ms, e0, e1));
    HIP_OK(hipEventDestroy(e0));
    HIP_OK(hipEventDestroy(e1));
    return ms / reps;
}

const char *shape_name(int t) {
    static const char *n[kNumShapes] = {"64x64", "128x32", "32x128", "128x128",
                                        "64x64k16", "128x32k16", "64x64k8", "128x32k8",
                                        "128x32dma", "64x64dma", "32x128dma"};
    return n[t];
}

// Times every allowed tile shape of stage 1 and of stage 3 (with its split-K
// reduction) on the operator's buffers and keeps the fastest of each.
void tune_heff(pdmrg_ctx *ctx, pdmrg_heff *op, const std::string &key) {
    hipStream_t s = ctx->stream;
    HeffPlan &pl = op->plan;
    const GemmPrec gp = gemm_prec(op->prec);
    const bool f64 = op->prec == PDMRG_F64;
    const size_t es = f64 ? sizeof(double) : sizeof(float);
    DevBuf xin(std::max<int64_t>(op->nX, 1) * es), yout(std::max<int64_t>(op->nX, 1) * sizeof(double));
    HIP_OK(hipMemsetAsync(xin.ptr, 0, xin.bytes, s));
    Slots sl{};
    sl.p[0] = xin.ptr;
    sl.p[1] = yout.ptr;
    sl.p[2] = op->lp;
    sl.p[3] = op->rp;
    sl.p[4] = op->t1;
    sl.p[5] = op->t2;
    const int reps = 3;
    int best1 = (int)pl.g1.shape, best3 = (int)pl.g3.shape;
    double t1best = 1e30, t3best = 1e30;
    std::ostringstream log;
    for (int t = 0; t < kNumShapes; ++t) {
        if (!(pl.g1.shapes_allowed & (1u << t))) continue;
        pl.set_g1_shape((TileShape)t, s);
        const double ms = time_ms(s, reps, [&] { pl.g1.launch(gp, f64, sl, s); });
        log << " g1 " << shape_name(t) << ' ' << ms;
        if (ms < t1best) { t1best = ms; best1 = t; }
    }
    const size_t pes = f64 ? sizeof(double) : sizeof(float);   // partial element size
    int parts3 = pl.parts3;
    for (int t = 0; t < kNumShapes; ++t) {
        if (!(pl.g3.shapes_allowed & (1u << t))) continue;
        // split-K factors: the default one and the others that still give >= 256 tiles
        const int tiles = std::max(1, pl.g3_base.ntiles_for((TileShape)t));
        std::vector<int> cand = {pl.default_parts((TileShape)t)};
        for (int p : {1, 2, 3, 4, 6, 8})
            if (p != cand[0] && tiles * p >= 256) cand.push_back(p);
        for (int parts : cand) {
            pl.set_g3_shape((TileShape)t, s, parts);
            op->P.ensure(std::max<int64_t>(pl.nP, 1) * pes);
            op->pp = op->P.ptr;
            sl.p[6] = op->pp;
            const double ms = time_ms(s, reps, [&] {
                pl.g3.launch(gp, f64, sl, s);
                if (f64) pl.r3.launch(true, sl, s);
                else pl.r3.launch_f32_to_f64(sl, s);
            });
            log << " g3 " << shape_name(t) << "/" << parts << ' ' << ms;
            if (ms < t3best) { t3best = ms; best3 = t; parts3 = parts; }
        }
    }
    pl.set_g1_shape((TileShape)best1, s);
    pl.set_g3_shape((TileShape)best3, s, parts3);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache()[key] = Tuned{best1, best3, parts3};
    }
    if (ctx->autotune >= 2)
        std::fprintf(stderr, "pdmrg autotune: g1 %s g3 %s/%d  (ms:%s)\n", shape_name(best1), shape_name(best3),
                     parts3, log.str().c_str());
}
}  // namespace

// Bytes behind an operator's intermediate (1 T1, 2 T2, 3 split-K partials).
static size_t ws_bytes(const pdmrg_heff *o, int which) {
    const size_t es = o->prec == PDMRG_F64 ? sizeof(double) : sizeof(float);
    const HeffPlan &pl = o->plan;
    const int64_t n = which == 1 ? pl.nT1 : which == 2 ? pl.nT2 : pl.nP;
    return (size_t)std::max<int64_t>(n, 1) * es;
}

GemmPrec gemm_prec(int prec) {
    switch (prec) {
        case PDMRG_F64: return GemmPrec::F64;
        case PDMRG_F32: return GemmPrec::F32;
        case PDMRG_BF16X3: return GemmPrec::BF16X3;
    }
    throw Error(PDMRG_EINVAL, "unknown precision " + std::to_string(prec));
}

void heff_build(pdmrg_ctx *ctx, pdmrg_heff *op, const Bond &bl, const Bond &br, const Phys &p,
                const MpoSite &W1, const MpoSite &W2, const double *L, const double *R, int prec, bool may_time,
                bool borrow_env, const pdmrg_heff *ws_from) {
    hipStream_t s = ctx->stream;
    (void)gemm_prec(prec);
    op->prec = prec;
    op->plan.build(bl, br, p, W1, W2, prec, s);
    HeffPlan &pl = op->plan;
    op->nX = pl.X.size;
    op->nL = pl.Lt.size;
    op->nR = pl.Rt.size;
    // diagonal preconditioner from the FP64 environments
    op->diag.ensure(std::max<int64_t>(op->nX, 1) * sizeof(double));
    upload(op->diag_terms, pl.diag_terms, s);
    upload(op->diag_groups, pl.diag_groups, s);
    {
        Slots sl{};
        sl.p[0] = op->diag.ptr;
        sl.p[1] = L;
        sl.p[2] = R;
        launch_diag_terms(sl, op->diag_terms.as<DiagTerm>(), op->diag_groups.as<int32_t>(),
                          (int)pl.diag_groups.size() - 1, pl.diag_max_rows, s);
    }
    const size_t es = prec == PDMRG_F64 ? sizeof(double) : sizeof(float);
    if (prec == PDMRG_F64 && borrow_env) {
        op->lp = L;
        op->rp = R;
    } else {
        op->L.ensure(std::max<int64_t>(op->nL, 1) * es);
        op->R.ensure(std::max<int64_t>(op->nR, 1) * es);
        if (prec == PDMRG_F64) {
            if (op->nL) HIP_OK(hipMemcpyAsync(op->L.ptr, L, op->nL * es, hipMemcpyDeviceToDevice, s));
            if (op->nR) HIP_OK(hipMemcpyAsync(op->R.ptr, R, op->nR * es, hipMemcpyDeviceToDevice, s));
        } else if (prec == PDMRG_BF16X3) {   // split once per operator
            launch_convert_f64_split(L, op->L.as<uint32_t>(), op->nL, s);
            launch_convert_f64_split(R, op->R.as<uint32_t>(), op->nR, s);
        } else {
            launch_convert_f64_f32(L, op->L.as<float>(), op->nL, s);
            launch_convert_f64_f32(R, op->R.as<float>(), op->nR, s);
        }
        op->lp = op->L.ptr;
        op->rp = op->R.ptr;
    }
    if (prec != PDMRG_F64) op->xs.ensure(std::max<int64_t>(op->nX, 1) * sizeof(float));
    // intermediates: another operator's where they are large enough
    auto pick = [&](DevBuf &own, void *other, size_t other_bytes, size_t need) -> void * {
        if (other && other_bytes >= need) return other;
        own.ensure(need);
        return own.ptr;
    };
    const size_t n1 = std::max<int64_t>(pl.nT1, 1) * es, n2 = std::max<int64_t>(pl.nT2, 1) * es;
    op->t1 = pick(op->T1, ws_from ? ws_from->t1 : nullptr, ws_from ? ws_bytes(ws_from, 1) : 0, n1);
    op->t2 = pick(op->T2, ws_from ? ws_from->t2 : nullptr, ws_from ? ws_bytes(ws_from, 2) : 0, n2);
    if (ctx->autotune > 0) {
        const std::string key = tune_key(ctx->device, prec, bl, br, W1, W2);
        Tuned hit;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = tune_cache().find(key);
            if (it != tune_cache().end()) hit = it->second;
        }
        if (hit.shape1 >= 0) {
            if (hit.shape1 != (int)pl.g1.shape) pl.set_g1_shape((TileShape)hit.shape1, s);
            if (hit.shape3 != (int)pl.g3.shape || hit.parts3 != pl.parts3)
                pl.set_g3_shape((TileShape)hit.shape3, s, hit.parts3);
        } else if (may_time) {
            tune_heff(ctx, op, key);
        }
    }
    op->pp = pick(op->P, ws_from ? ws_from->pp : nullptr, ws_from ? ws_bytes(ws_from, 3) : 0,
                  std::max<int64_t>(pl.nP, 1) * (prec == PDMRG_F64 ? sizeof(double) : sizeof(float)));
}

int tune_export(const char *path) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    FILE *f = std::fopen(path, "w");
    PD_REQUIRE(f != nullptr, PDMRG_EINVAL, std::string("autotune export: cannot write ") + path);
    int n = 0;
    for (const auto &kv : tune_cache()) {
        std::fprintf(f, "%s\t%d\t%d\t%d\n", kv.first.c_str(), kv.second.shape1, kv.second.shape3, kv.second.parts3);
        ++n;
    }
    std::fclose(f);
    return n;
}

int tune_import(const char *path) {
    FILE *f = std::fopen(path, "r");
    PD_REQUIRE(f != nullptr, PDMRG_EINVAL, std::string("autotune import: cannot read ") + path);
    std::vector<std::pair<std::string, Tuned>> rows;
    char line[1 << 14];
    while (std::fgets(line, sizeof line, f)) {
        std::string l(line);
        while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
        if (l.empty()) continue;
        const size_t t3 = l.rfind('\t'), t2 = l.rfind('\t', t3 - 1), t1 = l.rfind('\t', t2 - 1);
        if (t1 == std::string::npos || t2 == std::string::npos || t3 == std::string::npos) {
            std::fclose(f);
            throw Error(PDMRG_EINVAL, "autotune import: malformed line in " + std::string(path));
        }
        Tuned t;
        t.shape1 = std::atoi(l.c_str() + t1 + 1);
        t.shape3 = std::atoi(l.c_str() + t2 + 1);
        t.parts3 = std::atoi(l.c_str() + t3 + 1);
        if (t.shape1 < 0 || t.shape1 >= kNumShapes || t.shape3 < 0 || t.shape3 >= kNumShapes || t.parts3 < 1 ||
            t.parts3 > 8) {
            std::fclose(f);
            throw Error(PDMRG_EINVAL, "autotune import: entry out of range in " + std::string(path));
        }
        rows.push_back({l.substr(0, t1), t});
    }
    std::fclose(f);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (auto &r : rows) tune_cache()[r.first] = r.second;
    return (int)rows.size();
}

void grad_site_run(pdmrg_ctx *ctx, const GradPlan &plan, const double *L, const double *psi, const double *R,
                   double *G) {
    const size_t nU1 = std::max<int64_t>(plan.nU1, 1), nZ = std::max<int64_t>(plan.nZ, 1);
    const size_t np = std::max<size_t>(plan.dtiles.size(), 1);
    ctx->ws_grad.ensure((nU1 + nZ + np) * sizeof(double));
    double *U1 = ctx->ws_grad.as<double>();
    plan.run(L, psi, R, U1, U1 + nU1, U1 + nU1 + nZ, G, ctx->stream);
}

// The kernels of one product on stream s (no memset or copy nodes, so the
// sequence can be captured into a graph).
static void heff_launch(pdmrg_heff *op, const double *x, double *y, hipStream_t s, hipEvent_t *ev) {
    const HeffPlan &pl = op->plan;
    const GemmPrec gp = gemm_prec(op->prec);
    const bool f64 = op->prec == PDMRG_F64;
    Slots sl{};
    if (ev) HIP_OK(hipEventRecord(ev[0], s));
    if (f64) {
        sl.p[0] = x;
    } else {
        if (op->prec == PDMRG_BF16X3) launch_convert_f64_split(x, op->xs.as<uint32_t>(), op->nX, s);
        else launch_convert_f64_f32(x, op->xs.as<float>(), op->nX, s);
        sl.p[0] = op->xs.ptr;
    }
    sl.p[1] = y;
    sl.p[2] = op->lp;
    sl.p[3] = op->rp;
    sl.p[4] = op->t1;
    sl.p[5] = op->t2;
    sl.p[6] = op->pp;
    pl.g1.launch(gp, f64, sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[1], s));
    if (op->prec == PDMRG_BF16X3) pl.w.launch_split(sl, s);   // T2 is stage 3's split A operand
    else pl.w.launch(f64, sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[2], s));
    pl.g3.launch(gp, f64, sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[3], s));
    if (f64) pl.r3.launch(true, sl, s);
    else pl.r3.launch_f32_to_f64(sl, s);
    if (ev) HIP_OK(hipEventRecord(ev[4], s));
}

void heff_run(pdmrg_ctx *ctx, pdmrg_heff *op, const double *x, double *y) {
    hipStream_t s = ctx->stream;
    if (ctx->timing) {
        const size_t need = (size_t)(ctx->n_timed + 1) * kTimingEvents;
        while (ctx->ev_pool.size() < need) {
            hipEvent_t e;
            HIP_OK(hipEventCreate(&e));
            ctx->ev_pool.push_back(e);
        }
        hipEvent_t *ev = &ctx->ev_pool[(size_t)ctx->n_timed * kTimingEvents];
        ctx->n_timed += 1;
        heff_launch(op, x, y, s, ev);
        return;
    }
    if (!ctx->graphs) {
        heff_launch(op, x, y, s, nullptr);
        return;
    }
    // graph replay: one captured kernel sequence per (x, y) pair
    for (auto &gr : op->graphs)
        if (gr.x == x && gr.y == y) {
            HIP_OK(hipGraphLaunch(gr.exec, s));
            return;
        }
    if (op->graphs.size() >= pdmrg_heff::kMaxGraphs) {
        heff_launch(op, x, y, s, nullptr);
        return;
    }
    if (!ctx->cap_stream) HIP_OK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    pdmrg_heff::Graph gr;
    gr.x = x;
    gr.y = y;
    HIP_OK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        heff_launch(op, x, y, ctx->cap_stream, nullptr);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(ctx->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    HIP_OK(hipStreamEndCapture(ctx->cap_stream, &gr.graph));
    HIP_OK(hipGraphInstantiate(&gr.exec, gr.graph, nullptr, nullptr, 0));
    op->graphs.push_back(gr);
    HIP_OK(hipGraphLaunch(gr.exec, s));
}

}  // namespace pdmrg
