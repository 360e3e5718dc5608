// Builders of the contraction work lists (host bookkeeping).
#include "plans.hpp"

namespace pdmrg {

int GemmList::add_item(int c_slot, int64_t c_off, int M, int N, int ldc) {
    GemmItem it{};
    it.c_off = c_off;
    it.c_slot = c_slot;
    it.M = M;
    it.N = N;
    it.ldc = ldc;
    it.seg0 = (int32_t)segs.size();
    it.nseg = 0;
    it.rmap = -1;
    items.push_back(it);
    blk0.push_back(-1);
    return (int)items.size() - 1;
}

int GemmList::add_stacked_item(int c_slot, int N, const std::vector<RowBlock> &blks) {
    PD_REQUIRE(!blks.empty(), PDMRG_EINVAL, "gemm list: stacked item without blocks");
    GemmItem it{};
    it.c_off = 0;
    it.c_slot = c_slot;
    it.N = N;
    it.ldc = N;
    it.seg0 = (int32_t)segs.size();
    it.nseg = 0;
    it.rmap = (int32_t)rowoff.size();
    blk0.push_back((int32_t)blocks.size());
    int M = 0;
    for (RowBlock b : blks) {
        PD_REQUIRE(b.rows > 0 && b.ldc >= N, PDMRG_EINVAL, "gemm list: bad stacked block");
        b.r0 = M;
        for (int r = 0; r < b.rows; ++r) rowoff.push_back(b.c_off + (int64_t)r * b.ldc);
        blocks.push_back(b);
        M += b.rows;
    }
    blocks.push_back(RowBlock{0, M, 0, 0});   // terminator: r0 = M
    it.M = M;
    items.push_back(it);
    return (int)items.size() - 1;
}

void GemmList::add_seg(int a_slot, int64_t a_off, int lda, int b_slot, int64_t b_off, int ldb, int K) {
    PD_REQUIRE(!items.empty(), PDMRG_EINVAL, "gemm list: segment without item");
    GemmSeg sg{};
    sg.a_off = a_off;
    sg.b_off = b_off;
    sg.a_slot = a_slot;
    sg.b_slot = b_slot;
    sg.K = K;
    sg.lda = lda;
    sg.ldb = ldb;
    segs.push_back(sg);
    GemmItem &it = items.back();
    it.nseg += 1;
    flops += 2.0 * it.M * (double)it.N * K;
}

static int64_t item_k(const GemmList &g, const GemmItem &it) {
    int64_t k = 0;
    for (int j = 0; j < it.nseg; ++j) k += g.segs[it.seg0 + j].K;
    return k;
}

int GemmList::ntiles_for(TileShape t) const {
    const int bm = tile_bm(t), bn = tile_bn(t);
    int n = 0;
    for (const GemmItem &it : items) n += ((it.M + bm - 1) / bm) * ((it.N + bn - 1) / bn);
    return n;
}

double GemmList::padded_flops(TileShape t) const {
    const int bm = tile_bm(t), bn = tile_bn(t);
    double f = 0.0;
    for (const GemmItem &it : items)
        f += 2.0 * ((it.M + bm - 1) / bm * bm) * (double)((it.N + bn - 1) / bn * bn) * (double)item_k(*this, it);
    return f;
}

void GemmList::pick_tile() {
    // Relative throughput per padded flop of each shape, from timings of the
    // H_eff GEMMs of the 8 x 4 cylinder (m = 1024) on MI355X: shorter K steps
    // (more resident workgroups) win on these short, ragged K loops, and the
    // LDS-DMA shapes (FP32) ran 1.4-1.9x faster than their full-depth base
    // shapes (stage 1: 64x64 51.6 -> 36.4 us, 128x32 56.8 -> 38.5 us,
    // 32x128 70.6 -> 37.6 us).
    static const double kRate[kNumShapes] = {1.0, 1.0, 0.8, 0.75, 1.1, 1.15, 1.05, 1.2, 1.45, 1.45, 1.2};
    double best = 0.0;
    bool have = false;
    for (int t = 0; t < kNumShapes; ++t) {
        if (!(shapes_allowed & (1u << t))) continue;
        const TileShape ts = (TileShape)t;
        double cap = 0.0;   // tiles after the split-K the long items allow
        const int bm = tile_bm(ts), bn = tile_bn(ts);
        for (const GemmItem &it : items) {
            const double nt = ((it.M + bm - 1) / bm) * (double)((it.N + bn - 1) / bn);
            cap += nt * std::max<int64_t>(1, std::min<int64_t>(8, item_k(*this, it) / 256));
        }
        const double fill = std::min(1.0, cap / 1024.0);
        const double cost = padded_flops(ts) / (kRate[t] * std::max(fill, 1e-3));
        if (!have || cost < best * 0.999) {
            best = cost;
            shape = ts;
            have = true;
        }
    }
}

GemmList GemmList::host_copy() const {
    GemmList g;
    g.ta = ta;
    g.tb = tb;
    g.elem_bytes = elem_bytes;
    g.shape = shape;
    g.shapes_allowed = shapes_allowed;
    g.items = items;
    g.segs = segs;
    g.rowoff = rowoff;
    g.blk0 = blk0;
    g.blocks = blocks;
    g.flops = flops;
    return g;
}

// Launch order of the tiles.  Workgroup b of a launch runs on XCD b % 8 (the
// dispatcher deals workgroups to the 8 XCDs in turn) and tiles[b].  The tiles
// of an item are cut into chunks of consecutive rows, each about 1/128 of
// the launch's work (work = K + a fixed prologue/epilogue cost per tile), so an
// item, or a large item's row range, stays on one XCD and its L2 (the tiles
// of a row share the A panel, the rows of an item the B panel).  Chunks are
// dealt to XCDs largest first, each to the XCD of least work so far, then
// every XCD's list runs largest chunk first and the lists are interleaved;
// shorter lists are padded with idle tiles (item = -1).
static std::vector<GemmTile> place_tiles(const std::vector<GemmItem> &items, const std::vector<int64_t> &kof,
                                         int bm, int bn) {
    constexpr int kXcd = 8, kChunksPerXcd = 16;
    constexpr double kTileCost = 64.0;   // prologue + epilogue, in K units
    double total = 0.0;
    for (size_t i = 0; i < items.size(); ++i)
        if (items[i].M > 0 && items[i].N > 0)
            total += ((items[i].M + bm - 1) / bm) * (double)((items[i].N + bn - 1) / bn) * ((double)kof[i] + kTileCost);
    const double target = total / (kXcd * kChunksPerXcd);
    struct Chunk { int item, m_begin, m_end; double cost; };
    std::vector<Chunk> chunks;
    for (size_t i = 0; i < items.size(); ++i) {
        const GemmItem &it = items[i];
        if (it.M <= 0 || it.N <= 0) continue;
        const double row_cost = ((it.N + bn - 1) / bn) * ((double)kof[i] + kTileCost);
        Chunk c{(int)i, 0, 0, 0.0};
        for (int m0 = 0; m0 < it.M; m0 += bm) {
            c.m_end = std::min(m0 + bm, it.M);
            c.cost += row_cost;
            if (c.cost >= target) {
                chunks.push_back(c);
                c = Chunk{(int)i, c.m_end, c.m_end, 0.0};
            }
        }
        if (c.m_end > c.m_begin) chunks.push_back(c);
    }
    std::stable_sort(chunks.begin(), chunks.end(), [](const Chunk &a, const Chunk &b) { return a.cost > b.cost; });
    std::vector<std::vector<GemmTile>> lists(kXcd);
    double load[kXcd] = {};
    for (const Chunk &c : chunks) {
        const int x = (int)(std::min_element(load, load + kXcd) - load);
        load[x] += c.cost;
        for (int m0 = c.m_begin; m0 < c.m_end; m0 += bm)
            for (int n0 = 0; n0 < items[c.item].N; n0 += bn) lists[x].push_back(GemmTile{c.item, m0, n0, 0});
    }
    size_t len = 0;
    for (const auto &l : lists) len = std::max(len, l.size());
    std::vector<GemmTile> out(len * kXcd, GemmTile{-1, 0, 0, 0});
    for (int x = 0; x < kXcd; ++x)
        for (size_t j = 0; j < lists[x].size(); ++j) out[j * kXcd + x] = lists[x][j];
    return out;
}

void GemmList::finish(hipStream_t s) {
    build_tiles();
    upload(d_items, items, s);
    upload(d_segs, segs, s);
    upload(d_tiles, tiles, s);
    if (ftiles.empty()) d_ftiles.release();
    else upload(d_ftiles, ftiles, s);
    if (rowoff.empty()) d_rowoff.release();
    else upload(d_rowoff, rowoff, s);
}

void GemmList::build_tiles() {
    if (!(shapes_allowed & (1u << (int)shape)))
        shape = (shapes_allowed & (1u << (int)TileShape::T64x64)) ? TileShape::T64x64 : TileShape::T64x64_D;
    const int bm = tile_bm(shape), bn = tile_bn(shape);
    std::vector<int64_t> kof(items.size());
    ntiles_real = 0;
    for (size_t i = 0; i < items.size(); ++i) {
        kof[i] = item_k(*this, items[i]);
        if (items[i].M > 0 && items[i].N > 0)
            ntiles_real += ((items[i].M + bm - 1) / bm) * ((items[i].N + bn - 1) / bn);
    }
    tiles = place_tiles(items, kof, bm, bn);
    check_grid((int64_t)tiles.size(), 256, "gemm");
    PD_REQUIRE(std::count_if(tiles.begin(), tiles.end(), [](const GemmTile &t) { return t.item >= 0; }) ==
                   ntiles_real, PDMRG_ESHAPE, "gemm: tile placement lost tiles");
    ftiles.clear();
    bool single = !ta && !tb;
    for (const GemmItem &it : items) single = single && it.nseg <= 1;
    if (single && ((kDmaShapes >> (int)shape) & 1u)) {
        for (const GemmTile &t : tiles) {
            FlatTile f{};
            if (t.item >= 0) {
                const GemmItem &it = items[t.item];
                f.c_off = it.c_off;
                f.c_slot = f.a_slot = f.b_slot = it.c_slot;
                f.rmap = it.rmap;
                f.M = it.M;
                f.N = it.N;
                f.ldc = it.ldc;
                f.m0 = t.m0;
                f.n0 = t.n0;
                if (it.nseg == 1) {
                    const GemmSeg &sg = segs[it.seg0];
                    f.a_off = sg.a_off;
                    f.b_off = sg.b_off;
                    f.a_slot = sg.a_slot;
                    f.b_slot = sg.b_slot;
                    f.K = std::max(sg.K, 0);
                    f.lda = sg.lda;
                    f.ldb = sg.ldb;
                }
            }
            ftiles.push_back(f);
        }
    }
}

static void check_span(const std::vector<int64_t> &slot_elems, int slot, int64_t off, int rows, int cols,
                       int64_t ld, const char *what) {
    if (rows <= 0 || cols <= 0) return;
    PD_REQUIRE(slot >= 0 && slot < (int)slot_elems.size(), PDMRG_ESHAPE, std::string(what) + ": bad slot");
    PD_REQUIRE(ld >= cols, PDMRG_ESHAPE, std::string(what) + ": leading dimension below width");
    const int64_t last = off + (int64_t)(rows - 1) * ld + (cols - 1);
    PD_REQUIRE(off >= 0 && last < slot_elems[slot], PDMRG_ESHAPE,
               std::string(what) + ": work list reaches outside its buffer");
}

void GemmList::validate(const std::vector<int64_t> &slot_elems) const {
    for (const GemmItem &it : items) {
        if (it.rmap >= 0) {
            PD_REQUIRE(it.rmap + (int64_t)it.M <= (int64_t)rowoff.size(), PDMRG_ESHAPE, "gemm C: row map too short");
            for (int r = 0; r < it.M; ++r)
                check_span(slot_elems, it.c_slot, it.c_off + rowoff[it.rmap + r], 1, it.N, it.N, "gemm C row");
        } else {
            check_span(slot_elems, it.c_slot, it.c_off, it.M, it.N, it.ldc, "gemm C");
        }
        // buffer-load descriptors address one segment operand with 32-bit byte offsets
        for (int k = 0; k < it.nseg; ++k) {
            const GemmSeg &sg = segs[it.seg0 + k];
            const int64_t span_a = ta ? (int64_t)sg.K * sg.lda : (int64_t)it.M * sg.lda;
            const int64_t span_b = tb ? (int64_t)it.N * sg.ldb : (int64_t)sg.K * sg.ldb;
            PD_REQUIRE(span_a * elem_bytes < ((int64_t)1 << 31) && span_b * elem_bytes < ((int64_t)1 << 31),
                       PDMRG_ESHAPE,
                       "gemm: operand block exceeds 2 GiB");
        }
        for (int k = 0; k < it.nseg; ++k) {
            const GemmSeg &sg = segs[it.seg0 + k];
            if (ta) check_span(slot_elems, sg.a_slot, sg.a_off, sg.K, it.M, sg.lda, "gemm A^T");
            else check_span(slot_elems, sg.a_slot, sg.a_off, it.M, sg.K, sg.lda, "gemm A");
            if (tb) check_span(slot_elems, sg.b_slot, sg.b_off, it.N, sg.K, sg.ldb, "gemm B^T");
            else check_span(slot_elems, sg.b_slot, sg.b_off, sg.K, it.N, sg.ldb, "gemm B");
        }
    }
}

void LcList::validate(const std::vector<int64_t> &slot_elems) const {
    for (const LcTask &t : tasks) {
        PD_REQUIRE((int64_t)t.rows * t.cols < ((int64_t)1 << 31), PDMRG_ESHAPE, "W stage: block too large");
        // the kernel forms row * ld + col in 32 bits
        PD_REQUIRE(t.rows == 0 || (int64_t)(t.rows - 1) * t.ld + t.cols < ((int64_t)1 << 32), PDMRG_ESHAPE,
                   "W stage: block span too large");
        for (int j = 0; j < t.nsrc; ++j)
            PD_REQUIRE(t.rows == 0 || (int64_t)(t.rows - 1) * srcs[t.src0 + j].ld + t.cols < ((int64_t)1 << 32),
                       PDMRG_ESHAPE, "W stage: source span too large");
        check_span(slot_elems, t.dst_slot, t.dst_off, t.rows, t.cols, t.ld, "W stage dst");
        for (int j = 0; j < t.nsrc; ++j) {
            const LcSrc &sj = srcs[t.src0 + j];
            check_span(slot_elems, sj.slot, sj.off, t.rows, t.cols, sj.ld, "W stage src");
        }
    }
}

int64_t GemmList::split_k(int parts, int pslot, LcList &reduce, bool all) {
    if (parts <= 1 && !all) return 0;
    std::vector<GemmItem> nitems;
    std::vector<GemmSeg> nsegs;
    std::vector<int32_t> nblk0;
    std::vector<RowBlock> nblocks;
    int64_t pel = 0;
    // K range length of the longest item's parts; every item is cut into
    // ranges of about that length, so no tile's K loop is much longer than
    // another's (the longest tile bounds the launch), each range >= 64
    int64_t kmax = 0;
    for (const GemmItem &it : items) kmax = std::max(kmax, item_k(*this, it));
    const double krange = std::max(1.0, (double)kmax / std::max(parts, 1));
    for (size_t ii = 0; ii < items.size(); ++ii) {
        const GemmItem &it = items[ii];
        const int64_t ktot = item_k(*this, it);
        const int ip = (int)std::max<int64_t>(1, std::min<int64_t>({8, std::llround(ktot / krange), ktot / 64}));
        if (it.M == 0 || it.N == 0 || (ip == 1 && !all)) {
            GemmItem c = it;
            c.seg0 = (int32_t)nsegs.size();
            for (int k = 0; k < it.nseg; ++k) nsegs.push_back(segs[it.seg0 + k]);
            if (blk0[ii] >= 0) {
                nblk0.push_back((int32_t)nblocks.size());
                for (int b = blk0[ii];; ++b) {
                    nblocks.push_back(blocks[b]);
                    if (blocks[b].r0 == it.M && blocks[b].rows == 0) break;
                }
            } else {
                nblk0.push_back(-1);
            }
            nitems.push_back(c);
            continue;
        }
        // the output blocks this item writes: one plain block, or its stacked blocks
        std::vector<RowBlock> outb;
        if (blk0[ii] >= 0) {
            for (int b = blk0[ii]; blocks[b].rows > 0; ++b) outb.push_back(blocks[b]);
        } else {
            outb.push_back(RowBlock{it.c_off, 0, it.M, it.ldc});
        }
        const int64_t pbase = pel;
        for (int p = 0; p < ip; ++p) {
            // K range [kb, ke), boundaries rounded to multiples of 32
            const int64_t kb = (ktot * p / ip) / 32 * 32;
            const int64_t ke = p + 1 == ip ? ktot : (ktot * (p + 1) / ip) / 32 * 32;
            GemmItem c{};
            c.c_slot = pslot;
            c.c_off = pel;
            c.M = it.M;
            c.N = it.N;
            c.ldc = it.N;
            c.rmap = -1;
            c.seg0 = (int32_t)nsegs.size();
            c.nseg = 0;
            int64_t g0 = 0;   // global K index of the current segment's start
            for (int k = 0; k < it.nseg; ++k) {
                GemmSeg sg = segs[it.seg0 + k];
                const int64_t s0 = std::max<int64_t>(kb, g0), s1 = std::min<int64_t>(ke, g0 + sg.K);
                if (s1 > s0) {
                    const int64_t d = s0 - g0;
                    GemmSeg sub = sg;
                    sub.K = (int32_t)(s1 - s0);
                    sub.a_off += ta ? d * sg.lda : d;
                    sub.b_off += tb ? d : d * sg.ldb;
                    nsegs.push_back(sub);
                    c.nseg += 1;
                }
                g0 += sg.K;
            }
            nitems.push_back(c);
            nblk0.push_back(-1);
            pel += (int64_t)it.M * it.N;
        }
        // fixed-order reduction of the parts into each output block
        for (const RowBlock &ob : outb) {
            reduce.add_task(it.c_slot, ob.c_off, ob.rows, it.N, ob.ldc);
            for (int p = 0; p < ip; ++p)
                reduce.add_src(pslot, pbase + (int64_t)p * it.M * it.N + (int64_t)ob.r0 * it.N, it.N, 1.0);
        }
    }
    items.swap(nitems);
    segs.swap(nsegs);
    blk0.swap(nblk0);
    blocks.swap(nblocks);
    return pel;
}

void GemmList::launch(GemmPrec prec, bool c_is_f64, const Slots &sl, hipStream_t s) const {
    GemmDev dv{d_items.as<GemmItem>(), d_segs.as<GemmSeg>(), d_tiles.as<GemmTile>(), d_ftiles.as<FlatTile>(),
               d_rowoff.as<int64_t>()};
    launch(prec, c_is_f64, sl, dv, s);
}

void GemmList::launch(GemmPrec prec, bool c_is_f64, const Slots &sl, const GemmDev &dv, hipStream_t s) const {
    PD_REQUIRE(prec != GemmPrec::BF16X3 || !ftiles.empty() || tiles.empty(), PDMRG_EINVAL,
               "gemm: BF16x3 needs an LDS-DMA plan (split operands)");
    if (!ftiles.empty()) {
        launch_gemm_flat(prec, shape, c_is_f64, sl, dv.ftiles, dv.rowoff, (int)ftiles.size(), s);
        return;
    }
    launch_gemm(prec, shape, ta, tb, c_is_f64, sl, dv.items, dv.segs, dv.tiles, dv.rowoff, (int)tiles.size(), s);
}

int LcList::add_task(int dst_slot, int64_t dst_off, int rows, int cols, int ld) {
    LcTask t{};
    t.dst_off = dst_off;
    t.dst_slot = dst_slot;
    t.rows = rows;
    t.cols = cols;
    t.ld = ld;
    t.src0 = (int32_t)srcs.size();
    t.nsrc = 0;
    tasks.push_back(t);
    elems_out += (int64_t)rows * cols;
    return (int)tasks.size() - 1;
}

void LcList::add_src(int slot, int64_t off, int ld, double coef) {
    LcSrc sj{};
    sj.off = off;
    sj.slot = slot;
    sj.ld = ld;
    sj.coef = coef;
    srcs.push_back(sj);
    LcTask &t = tasks.back();
    t.nsrc += 1;
    flops += 2.0 * t.rows * (double)t.cols;
    elems_in += (int64_t)t.rows * t.cols;
}

void LcList::build_tiles() {
    tiles.clear();
    for (size_t i = 0; i < tasks.size(); ++i) {
        const LcTask &t = tasks[i];
        const int64_t n = (int64_t)t.rows * t.cols;
        for (int64_t c = 0; c * chunk < n; ++c) tiles.push_back(LcTile{(int32_t)i, (int32_t)c, chunk, 0});
    }
}

void LcList::finish(hipStream_t s) {
    build_tiles();
    upload(d_tasks, tasks, s);
    upload(d_srcs, srcs, s);
    upload(d_tiles, tiles, s);
}

void LcList::launch_f32_to_f64(const Slots &sl, hipStream_t s) const {
    launch_lincomb_f32_f64(chunk, sl, d_tasks.as<LcTask>(), d_srcs.as<LcSrc>(), d_tiles.as<LcTile>(),
                           (int)tiles.size(), s);
}

void LcList::launch_split(const Slots &sl, hipStream_t s) const {
    launch_lincomb_split(chunk, sl, d_tasks.as<LcTask>(), d_srcs.as<LcSrc>(), d_tiles.as<LcTile>(), (int)tiles.size(),
                         s);
}

void LcList::launch(bool f64, const Slots &sl, hipStream_t s) const {
    launch(f64, sl, LcDev{d_tasks.as<LcTask>(), d_srcs.as<LcSrc>(), d_tiles.as<LcTile>()}, s);
}

void LcList::launch(bool f64, const Slots &sl, const LcDev &dv, hipStream_t s) const {
    launch_lincomb(f64, chunk, sl, dv.tasks, dv.srcs, dv.tiles, (int)tiles.size(), s);
}

std::vector<double> two_site_mpo(const MpoSite &W1, const MpoSite &W2) {
    // W12[w][s1][t1][s2][t2][w2] = sum_c W1[w][s1][t1][c] W2[c][s2][t2][w2]
    PD_REQUIRE(W1.Dr == W2.Dl && W1.d == W2.d, PDMRG_ESHAPE, "two-site MPO: inner channel mismatch");
    const int d = W1.d, Dl = W1.Dl, Dm = W1.Dr, Dr = W2.Dr;
    std::vector<double> W12((size_t)Dl * d * d * d * d * Dr, 0.0);
    for (int w = 0; w < Dl; ++w)
        for (int s1 = 0; s1 < d; ++s1)
            for (int t1 = 0; t1 < d; ++t1)
                for (int c = 0; c < Dm; ++c) {
                    const double a = W1.at(w, s1, t1, c);
                    if (a == 0.0) continue;
                    for (int s2 = 0; s2 < d; ++s2)
                        for (int t2 = 0; t2 < d; ++t2)
                            for (int w2 = 0; w2 < Dr; ++w2) {
                                const double b = W2.at(c, s2, t2, w2);
                                if (b == 0.0) continue;
                                W12[((((((size_t)w * d + s1) * d + t1) * d + s2) * d + t2) * Dr) + w2] += a * b;
                            }
                }
    return W12;
}

// ---------------------------------------------------------------- H_eff
void HeffPlan::build(const Bond &bl_, const Bond &br_, const Phys &p_, const MpoSite &W1, const MpoSite &W2,
                     int prec, hipStream_t s) {
    bl = bl_;
    br = br_;
    p = p_;
    const int d = p.d(), d2 = d * d;
    PD_REQUIRE(W1.d == d && W2.d == d, PDMRG_ESHAPE, "heff: MPO local dimension mismatch");
    PD_REQUIRE(W1.Dr == W2.Dl, PDMRG_ESHAPE, "heff: W1/W2 channel mismatch");
    const int Dl = W1.Dl, Dr = W2.Dr;
    X = two_site_layout(bl, br, p);
    Lt = env_l_layout(bl, W1.dl);
    Rt = env_r_layout(br, W2.dr);
    const std::vector<double> W12 = two_site_mpo(W1, W2);
    auto w12 = [&](int w, int s1, int t1, int s2, int t2, int w2) {
        return W12[((((((size_t)w * d + s1) * d + t1) * d + s2) * d + t2) * Dr) + w2];
    };
    const int nl = bl.nsec();

    // stage 1: T1[j] = Lket[j] (rows (w, a)) x X[j] (rows a', cols (t1 t2 b'))
    std::vector<int64_t> t1base(nl, -1);
    nT1 = 0;
    g1 = GemmList();
    g1.elem_bytes = prec == PDMRG_F64 ? 8 : 4;
    for (int j = 0; j < nl; ++j) {
        const int M = Lt.rows[j], N = X.cols[j], K = bl.dim[j];
        if (M == 0 || N == 0) continue;
        t1base[j] = nT1;
        g1.add_item(4, nT1, M, N, N);
        g1.add_seg(2, Lt.base[j], K, 0, X.base[j], N, K);
        nT1 += (int64_t)M * N;
    }

    // T2 blocks: one per output block (i, s1 s2) -> [dim(q_i) x Rt.rows[k]],
    // grouped by the bra sector k they multiply, so that the blocks sharing
    // R[k] form one contiguous (sum of dims) x Rt.rows[k] matrix.
    std::vector<int64_t> t2base((size_t)nl * d2, -1);
    std::vector<std::vector<std::pair<int, int>>> by_k(br.nsec());
    for (int i = 0; i < nl; ++i)
        for (int sg = 0; sg < d2; ++sg) {
            if (X.colo[(size_t)i * d2 + sg] < 0) continue;
            by_k[br.find(bl.q[i] + p.q[sg / d] + p.q[sg % d])].push_back({i, sg});
        }
    nT2 = 0;
    for (int k = 0; k < br.nsec(); ++k)
        for (auto [i, sg] : by_k[k]) {
            t2base[(size_t)i * d2 + sg] = nT2;
            nT2 += (int64_t)bl.dim[i] * Rt.rows[k];
        }

    // stage 2: W stage
    w = LcList();
    for (int i = 0; i < nl; ++i)
        for (int sg = 0; sg < d2; ++sg) {
            const int64_t tb = t2base[(size_t)i * d2 + sg];
            if (tb < 0) continue;
            const int s1 = sg / d, s2 = sg % d;
            const int qb = bl.q[i] + p.q[s1] + p.q[s2];
            const int k = br.find(qb);
            for (int w2 = 0; w2 < Dr; ++w2) {
                const int ro = Rt.rowo[(size_t)k * Dr + w2];
                if (ro < 0) continue;
                const int cols = br.dim_of(qb - W2.dr[w2]);
                w.add_task(5, tb + ro, bl.dim[i], cols, Rt.rows[k]);
                for (int ww = 0; ww < Dl; ++ww) {
                    const int j = bl.find(bl.q[i] - W1.dl[ww]);
                    if (j < 0 || t1base[j] < 0) continue;
                    const int lro = Lt.rowo[(size_t)j * Dl + ww];
                    if (lro < 0) continue;
                    for (int t1 = 0; t1 < d; ++t1)
                        for (int t2 = 0; t2 < d; ++t2) {
                            const double c = w12(ww, s1, t1, s2, t2, w2);
                            if (c == 0.0) continue;
                            const int co = X.colo[(size_t)j * d2 + t1 * d + t2];
                            if (co < 0) continue;
                            PD_REQUIRE(X.width[(size_t)j * d2 + t1 * d + t2] == cols, PDMRG_ESHAPE,
                                       "heff: MPO entry violates charge conservation");
                            w.add_src(4, t1base[j] + (int64_t)lro * X.cols[j] + co, X.cols[j], c);
                        }
                }
            }
        }

    // stage 3: y[i, s1 s2] = T2[i, s1 s2] x Rbra[k], one stacked item per k
    // (cut into several where the stacked T2 operand would span 2 GiB or
    // more, the reach of the kernels' 32-bit buffer offsets)
    g3 = GemmList();
    const int64_t es3 = prec == PDMRG_F64 ? 8 : 4;
    g3.elem_bytes = (int)es3;
    for (int k = 0; k < br.nsec(); ++k) {
        if (by_k[k].empty()) continue;
        const int64_t ld = std::max(Rt.rows[k], 1);
        size_t b0 = 0;
        while (b0 < by_k[k].size()) {
            std::vector<RowBlock> blks;
            int64_t rows = 0;
            size_t b1 = b0;
            for (; b1 < by_k[k].size(); ++b1) {
                const auto [i, sg] = by_k[k][b1];
                if (!blks.empty() && (rows + bl.dim[i]) * ld * es3 >= (int64_t(1) << 31)) break;
                blks.push_back(RowBlock{X.base[i] + X.colo[(size_t)i * d2 + sg], 0, bl.dim[i], X.cols[i]});
                rows += bl.dim[i];
            }
            g3.add_stacked_item(1, br.dim[k], blks);
            const auto [i0, sg0] = by_k[k][b0];
            if (Rt.rows[k] > 0)
                g3.add_seg(5, t2base[(size_t)i0 * d2 + sg0], Rt.rows[k], 3, Rt.base[k], br.dim[k], Rt.rows[k]);
            b0 = b1;
        }
    }

    // diag(H_eff): sum over channels with delta = 0 of L[a,w,a] W12 R[b,w2,b]
    diag_terms.clear();
    diag_groups.assign(1, 0);
    diag_max_rows = 0;
    for (int i = 0; i < nl; ++i)
        for (int sg = 0; sg < d2; ++sg) {
            if (X.colo[(size_t)i * d2 + sg] < 0) continue;
            const int s1 = sg / d, s2 = sg % d;
            const int k = br.find(bl.q[i] + p.q[s1] + p.q[s2]);
            DiagTerm base{};
            base.out_off = X.base[i] + X.colo[(size_t)i * d2 + sg];
            base.rows = bl.dim[i];
            base.cols = br.dim[k];
            base.ld = X.cols[i];
            diag_max_rows = std::max(diag_max_rows, base.rows);
            bool any = false;
            for (int ww = 0; ww < Dl; ++ww) {
                if (W1.dl[ww] != 0) continue;
                const int lro = Lt.rowo[(size_t)i * Dl + ww];
                if (lro < 0) continue;
                for (int w2 = 0; w2 < Dr; ++w2) {
                    if (W2.dr[w2] != 0) continue;
                    const double c = w12(ww, s1, s1, s2, s2, w2);
                    if (c == 0.0) continue;
                    const int rro = Rt.rowo[(size_t)k * Dr + w2];
                    if (rro < 0) continue;
                    DiagTerm t = base;
                    t.coef = c;
                    t.l_off = Lt.base[i] + (int64_t)lro * Lt.cols[i];
                    t.lstride = Lt.cols[i] + 1;
                    t.r_off = Rt.base[k] + (int64_t)rro * Rt.cols[k];
                    t.rstride = Rt.cols[k] + 1;
                    diag_terms.push_back(t);
                    any = true;
                }
            }
            if (!any) {   // still write zeros
                DiagTerm t = base;
                t.coef = 0.0;
                t.l_off = 0;
                t.r_off = 0;
                t.lstride = 0;
                t.rstride = 0;
                diag_terms.push_back(t);
            }
            diag_groups.push_back((int32_t)diag_terms.size());
        }

    // tile shapes: both lists are non-transposed with one segment per item,
    // so the LDS-DMA shapes apply; BF16x3 (split operands) runs only those
    if (prec == PDMRG_BF16X3) {
        g1.shapes_allowed = g3.shapes_allowed = kDmaShapes;
    } else {
        g1.shapes_allowed |= kDmaShapes;
        g3.shapes_allowed |= kDmaShapes;
    }
    for (GemmList *g : {&g1, &g3}) {
        // the cost model keeps FP64 on the register-staged kernel, which measured
        // faster than the LDS-DMA one in FP64 (the autotuner still times both)
        const unsigned all = g->shapes_allowed;
        if (prec == PDMRG_F64) g->shapes_allowed &= ~kDmaShapes;
        g->pick_tile();
        g->shapes_allowed = all;
    }
    const std::vector<int64_t> sz = {X.size, X.size, Lt.size, Rt.size, nT1, nT2, 0};
    g1.validate(sz);
    w.validate(sz);
    g1.finish(s);
    w.finish(s);
    g3_base = g3.host_copy();
    lowp = prec != PDMRG_F64;
    set_g3_shape(g3.shape, s);
}

void HeffPlan::set_g1_shape(TileShape t, hipStream_t s) {
    g1.shape = t;
    g1.finish(s);
}

int HeffPlan::default_parts(TileShape t) const {
    // split-K for stage 3: aim at >= 1024 output tiles (4 per CU)
    const int tiles3 = std::max(1, g3_base.ntiles_for(t));
    return std::max(1, std::min(8, (1024 + tiles3 - 1) / tiles3));
}

void HeffPlan::set_g3_shape(TileShape t, hipStream_t s, int parts) {
    g3 = g3_base.host_copy();
    g3.shape = t;
    if (parts <= 0) parts = default_parts(t);
    r3 = LcList();
    r3.chunk = kLcChunkSmall;
    // low precision: every item goes through the FP32 partial buffer and the
    // reduction writes the FP64 output
    nP = g3.split_k(parts, 6, r3, lowp);
    parts3 = parts;
    const std::vector<int64_t> sz = {X.size, X.size, Lt.size, Rt.size, nT1, nT2, nP};
    g3.validate(sz);
    r3.validate(sz);
    g3.finish(s);
    r3.finish(s);
}

// ---------------------------------------------------------------- environments
void EnvPlan::build(int dir_, const Bond &bl_, const Bond &br_, const Phys &p_, const MpoSite &W, hipStream_t s,
                    bool upload) {
    dir = dir_;
    bl = bl_;
    br = br_;
    p = p_;
    const int d = p.d();
    PD_REQUIRE(W.d == d, PDMRG_ESHAPE, "env: MPO local dimension mismatch");
    const int Dl = W.Dl, Dr = W.Dr;
    S = site_layout(bl, br, p);
    const int nl = bl.nsec(), nr = br.nsec();
    g1 = GemmList();
    g3 = GemmList();
    w = LcList();
    if (dir > 0) {
        Ein = env_l_layout(bl, W.dl);
        Eout = env_l_layout(br, W.dr);
        Aux = env_r_layout(br, W.dr);     // column structure of U2 blocks
        // E1: U1[j] = Lket[j] x A[j]
        std::vector<int64_t> u1base(nl, -1);
        nU1 = 0;
        for (int j = 0; j < nl; ++j) {
            const int M = Ein.rows[j], N = S.cols[j], K = bl.dim[j];
            if (M == 0 || N == 0) continue;
            u1base[j] = nU1;
            g1.add_item(3, nU1, M, N, N);
            g1.add_seg(0, Ein.base[j], K, 1, S.base[j], N, K);
            nU1 += (int64_t)M * N;
        }
        // U2 blocks (i, s): [dim(q_i) x Aux.rows[k]]
        std::vector<int64_t> u2base((size_t)nl * d, -1);
        nU2 = 0;
        for (int i = 0; i < nl; ++i)
            for (int sp = 0; sp < d; ++sp) {
                if (S.colo[(size_t)i * d + sp] < 0) continue;
                const int k = br.find(bl.q[i] + p.q[sp]);
                u2base[(size_t)i * d + sp] = nU2;
                nU2 += (int64_t)bl.dim[i] * Aux.rows[k];
            }
        // E2: U2[(i,s)][a, (w', b')] = sum W[w,s,t,w'] U1[q_i - dl_w][(w,a), (t,b')]
        for (int i = 0; i < nl; ++i)
            for (int sp = 0; sp < d; ++sp) {
                const int64_t ub = u2base[(size_t)i * d + sp];
                if (ub < 0) continue;
                const int qb = bl.q[i] + p.q[sp];
                const int k = br.find(qb);
                for (int w2 = 0; w2 < Dr; ++w2) {
                    const int ro = Aux.rowo[(size_t)k * Dr + w2];
                    if (ro < 0) continue;
                    const int cols = br.dim_of(qb - W.dr[w2]);
                    w.add_task(4, ub + ro, bl.dim[i], cols, Aux.rows[k]);
                    for (int ww = 0; ww < Dl; ++ww) {
                        const int j = bl.find(bl.q[i] - W.dl[ww]);
                        if (j < 0 || u1base[j] < 0) continue;
                        const int lro = Ein.rowo[(size_t)j * Dl + ww];
                        if (lro < 0) continue;
                        for (int t = 0; t < d; ++t) {
                            const double c = W.at(ww, sp, t, w2);
                            if (c == 0.0) continue;
                            const int co = S.colo[(size_t)j * d + t];
                            if (co < 0) continue;
                            PD_REQUIRE(S.width[(size_t)j * d + t] == cols, PDMRG_ESHAPE,
                                       "env: MPO entry violates charge conservation");
                            w.add_src(3, u1base[j] + (int64_t)lro * S.cols[j] + co, S.cols[j], c);
                        }
                    }
                }
            }
        // E3: Lout[j'] rows (w', b) = sum_s A[(i,s)]^T U2[(i,s)][:, w' segment]
        g3.ta = true;
        for (int jp = 0; jp < nr; ++jp)
            for (int w2 = 0; w2 < Dr; ++w2) {
                const int ro = Eout.rowo[(size_t)jp * Dr + w2];
                if (ro < 0) continue;
                const int k = br.find(br.q[jp] + W.dr[w2]);
                g3.add_item(2, Eout.base[jp] + (int64_t)ro * br.dim[jp], br.dim[k], br.dim[jp], br.dim[jp]);
                for (int sp = 0; sp < d; ++sp) {
                    const int i = bl.find(br.q[k] - p.q[sp]);
                    if (i < 0) continue;
                    const int64_t ub = u2base[(size_t)i * d + sp];
                    if (ub < 0) continue;
                    const int aro = Aux.rowo[(size_t)k * Dr + w2];
                    g3.add_seg(1, S.base[i] + S.colo[(size_t)i * d + sp], S.cols[i], 4, ub + aro, Aux.rows[k],
                               bl.dim[i]);
                }
            }
    } else {
        Ein = env_r_layout(br, W.dr);
        Eout = env_r_layout(bl, W.dl);
        // F1: Z1[(k,s)] = Rbra[k] x B[(i,s)]^T, i = q_k - q_s
        std::vector<int64_t> z1base((size_t)nr * d, -1);
        nU1 = 0;
        g1.tb = true;
        for (int k = 0; k < nr; ++k)
            for (int sp = 0; sp < d; ++sp) {
                const int i = bl.find(br.q[k] - p.q[sp]);
                if (i < 0 || Ein.rows[k] == 0) continue;
                z1base[(size_t)k * d + sp] = nU1;
                g1.add_item(3, nU1, Ein.rows[k], bl.dim[i], bl.dim[i]);
                g1.add_seg(0, Ein.base[k], br.dim[k], 1, S.base[i] + S.colo[(size_t)i * d + sp], S.cols[i],
                           br.dim[k]);
                nU1 += (int64_t)Ein.rows[k] * bl.dim[i];
            }
        // Z2 blocks (i, w): [S.cols[i'] x dim(q_i)], i' = q_i - dl_w
        std::vector<int64_t> z2base((size_t)nl * Dl, -1);
        nU2 = 0;
        for (int i = 0; i < nl; ++i)
            for (int ww = 0; ww < Dl; ++ww) {
                const int ip = bl.find(bl.q[i] - W.dl[ww]);
                if (ip < 0 || S.cols[ip] == 0) continue;
                z2base[(size_t)i * Dl + ww] = nU2;
                nU2 += (int64_t)S.cols[ip] * bl.dim[i];
            }
        // F2: Z2[(i,w)][(s', b'), a] = sum W[w,s,s',w2] Z1[(k,s)][(w2,b'), a]
        for (int i = 0; i < nl; ++i)
            for (int ww = 0; ww < Dl; ++ww) {
                const int64_t zb = z2base[(size_t)i * Dl + ww];
                if (zb < 0) continue;
                const int ip = bl.find(bl.q[i] - W.dl[ww]);
                for (int spp = 0; spp < d; ++spp) {
                    const int co = S.colo[(size_t)ip * d + spp];
                    if (co < 0) continue;
                    const int rows = S.width[(size_t)ip * d + spp];
                    w.add_task(4, zb + (int64_t)co * bl.dim[i], rows, bl.dim[i], bl.dim[i]);
                    for (int sp = 0; sp < d; ++sp) {
                        const int k = br.find(bl.q[i] + p.q[sp]);
                        if (k < 0) continue;
                        const int64_t z1 = z1base[(size_t)k * d + sp];
                        if (z1 < 0) continue;
                        for (int w2 = 0; w2 < Dr; ++w2) {
                            const double c = W.at(ww, sp, spp, w2);
                            if (c == 0.0) continue;
                            const int ro = Ein.rowo[(size_t)k * Dr + w2];
                            if (ro < 0) continue;
                            PD_REQUIRE(br.dim_of(br.q[k] - W.dr[w2]) == rows, PDMRG_ESHAPE,
                                       "env: MPO entry violates charge conservation");
                            w.add_src(3, z1 + (int64_t)ro * bl.dim[i], bl.dim[i], c);
                        }
                    }
                }
            }
        // F3: Rout[i] rows (w, a') = B[i'] x Z2[(i,w)]
        for (int i = 0; i < nl; ++i)
            for (int ww = 0; ww < Dl; ++ww) {
                const int ro = Eout.rowo[(size_t)i * Dl + ww];
                if (ro < 0) continue;
                const int ip = bl.find(bl.q[i] - W.dl[ww]);
                g3.add_item(2, Eout.base[i] + (int64_t)ro * bl.dim[i], bl.dim[ip], bl.dim[i], bl.dim[i]);
                const int64_t zb = z2base[(size_t)i * Dl + ww];
                if (zb >= 0) g3.add_seg(1, S.base[ip], S.cols[ip], 4, zb, bl.dim[i], S.cols[ip]);
            }
    }
    const std::vector<int64_t> sz = {Ein.size, S.size, Eout.size, nU1, nU2};
    g1.validate(sz);
    w.validate(sz);
    g3.validate(sz);
    g1.pick_tile();
    g3.pick_tile();
    if (!upload) return;
    g1.finish(s);
    w.finish(s);
    g3.finish(s);
}

void EnvPlan::run(GemmPrec prec, const void *env_in, const void *site, void *env_out, void *U1, void *U2,
                  const GemmDev &d1, const LcDev &dw, const GemmDev &d3, hipStream_t s) const {
    Slots sl{};
    sl.p[0] = env_in;
    sl.p[1] = site;
    sl.p[2] = env_out;
    sl.p[3] = U1;
    sl.p[4] = U2;
    const bool f64 = prec == GemmPrec::F64;
    g1.launch(prec, f64, sl, d1, s);
    w.launch(f64, sl, dw, s);
    g3.launch(prec, f64, sl, d3, s);
}

void EnvPlan::run(GemmPrec prec, const void *env_in, const void *site, void *env_out, void *U1, void *U2,
                  hipStream_t s) const {
    Slots sl{};
    sl.p[0] = env_in;
    sl.p[1] = site;
    sl.p[2] = env_out;
    sl.p[3] = U1;
    sl.p[4] = U2;
    const bool f64 = prec == GemmPrec::F64;
    g1.launch(prec, f64, sl, s);
    w.launch(f64, sl, s);
    g3.launch(prec, f64, sl, s);
}

// ---------------------------------------------------------------- gradient
void GradPlan::build(const Bond &bl_, const Bond &br_, const Phys &p_, const MpoSite &W, hipStream_t s) {
    bl = bl_;
    br = br_;
    p = p_;
    const int d = p.d();
    PD_REQUIRE(W.d == d, PDMRG_ESHAPE, "grad: MPO local dimension mismatch");
    Dl = W.Dl;
    Dr = W.Dr;
    S = site_layout(bl, br, p);
    Lt = env_l_layout(bl, W.dl);
    Rt = env_r_layout(br, W.dr);
    const int nl = bl.nsec();
    // stage 1: U1[j] = Lket[j] x psi[j]
    g1 = GemmList();
    std::vector<int64_t> u1base(nl, -1);
    nU1 = 0;
    for (int j = 0; j < nl; ++j) {
        const int M = Lt.rows[j], N = S.cols[j], K = bl.dim[j];
        if (M == 0 || N == 0) continue;
        u1base[j] = nU1;
        g1.add_item(3, nU1, M, N, N);
        g1.add_seg(0, Lt.base[j], K, 1, S.base[j], N, K);
        nU1 += (int64_t)M * N;
    }
    // stage 2: Z blocks [b'][b] = U1^T psi, then stage-3 dot tasks
    gz = GemmList();
    gz.ta = true;
    dots.clear();
    nZ = 0;
    for (int i = 0; i < nl; ++i)
        for (int w = 0; w < Dl; ++w) {
            const int j = bl.find(bl.q[i] - W.dl[w]);
            if (j < 0 || u1base[j] < 0) continue;
            const int lro = Lt.rowo[(size_t)j * Dl + w];
            if (lro < 0) continue;
            for (int sp = 0; sp < d; ++sp) {
                const int cs = S.colo[(size_t)i * d + sp];
                if (cs < 0) continue;
                const int qb = bl.q[i] + p.q[sp];
                const int kb = br.find(qb);
                for (int t = 0; t < d; ++t) {
                    const int ct = S.colo[(size_t)j * d + t];
                    if (ct < 0) continue;
                    const int qbk = bl.q[j] + p.q[t];
                    // channels w' of R with delta = qb - qbk
                    std::vector<int> wr;
                    for (int w2 = 0; w2 < Dr; ++w2)
                        if (W.dr[w2] == qb - qbk && Rt.rowo[(size_t)kb * Dr + w2] >= 0) wr.push_back(w2);
                    if (wr.empty()) continue;
                    const int M = br.dim_of(qbk), N = br.dim[kb], K = bl.dim[i];
                    gz.add_item(4, nZ, M, N, N);
                    gz.add_seg(3, u1base[j] + (int64_t)lro * S.cols[j] + ct, S.cols[j], 1, S.base[i] + cs, S.cols[i],
                               K);
                    for (int w2 : wr) {
                        const int64_t roff = Rt.base[kb] + (int64_t)Rt.rowo[(size_t)kb * Dr + w2] * br.dim[kb];
                        const int g = ((w * d + sp) * d + t) * Dr + w2;
                        dots.push_back(DotTask{nZ, roff, M * N, g});
                    }
                    nZ += (int64_t)M * N;
                }
            }
        }
    // dot tiles grouped by output entry, tasks of one entry in build order
    std::vector<int> order(dots.size());
    for (size_t k = 0; k < order.size(); ++k) order[k] = (int)k;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return dots[a].g < dots[b].g; });
    dtiles.clear();
    t0.clear();
    g_of.clear();
    for (size_t k = 0; k < order.size(); ++k) {
        const DotTask &dt = dots[order[k]];
        PD_REQUIRE(dt.n > 0, PDMRG_ESHAPE, "grad: empty block");
        if (g_of.empty() || g_of.back() != dt.g) {
            t0.push_back((int32_t)dtiles.size());
            g_of.push_back(dt.g);
        }
        for (int c = 0; c * kDotChunk < dt.n; ++c) dtiles.push_back(DotTile{order[k], c});
    }
    t0.push_back((int32_t)dtiles.size());
    for (const DotTask &dt : dots) {
        PD_REQUIRE(dt.a_off >= 0 && dt.a_off + dt.n <= nZ && dt.b_off >= 0 && dt.b_off + dt.n <= Rt.size,
                   PDMRG_ESHAPE, "grad: dot task outside its buffer");
        flops += 2.0 * dt.n;
    }
    flops += g1.flops + gz.flops;
    const std::vector<int64_t> sz = {Lt.size, S.size, Rt.size, nU1, nZ};
    g1.validate(sz);
    gz.validate(sz);
    g1.pick_tile();
    gz.pick_tile();
    g1.finish(s);
    gz.finish(s);
    upload(d_dots, dots, s);
    upload(d_dtiles, dtiles, s);
    upload(d_t0, t0, s);
    upload(d_gof, g_of, s);
}

void GradPlan::run(const double *L, const double *psi, const double *R, double *U1, double *Z, double *partial,
                   double *G, hipStream_t s) const {
    Slots sl{};
    sl.p[0] = L;
    sl.p[1] = psi;
    sl.p[2] = R;
    sl.p[3] = U1;
    sl.p[4] = Z;
    launch_fill(G, 0.0, (int64_t)Dl * p.d() * p.d() * Dr, s);
    g1.launch(GemmPrec::F64, true, sl, s);
    gz.launch(GemmPrec::F64, true, sl, s);
    launch_dot_partials(sl, 4, 2, d_dots.as<DotTask>(), d_dtiles.as<DotTile>(), (int)dtiles.size(), partial, s);
    launch_dot_reduce(partial, d_t0.as<int32_t>(), d_gof.as<int32_t>(), (int)g_of.size(), G, s);
}

// ---------------------------------------------------------------- merge
void MergePlan::build(const Bond &bl_, const Bond &bm_, const Bond &br_, const Phys &p_, hipStream_t s) {
    bl = bl_;
    bm = bm_;
    br = br_;
    p = p_;
    const int d = p.d(), d2 = d * d;
    SL = site_layout(bl, bm, p);
    SR = site_layout(bm, br, p);
    X = two_site_layout(bl, br, p);
    rs_base.clear();
    rs_vbase.clear();
    rs_rows.clear();
    rs_cols.clear();
    rs_max = 0;
    for (int k = 0; k < bm.nsec(); ++k) {
        if (SR.cols[k] == 0) continue;
        rs_base.push_back(SR.base[k]);
        rs_vbase.push_back(bm.off[k]);
        rs_rows.push_back(bm.dim[k]);
        rs_cols.push_back(SR.cols[k]);
        rs_max = std::max<int64_t>(rs_max, (int64_t)bm.dim[k] * SR.cols[k]);
    }
    g = GemmList();
    for (int i = 0; i < bl.nsec(); ++i)
        for (int s3 = 0; s3 < d; ++s3) {
            const int lco = SL.colo[(size_t)i * d + s3];
            if (lco < 0) continue;
            const int k = bm.find(bl.q[i] + p.q[s3]);
            if (SR.cols[k] == 0) continue;
            int col0 = -1;
            for (int s4 = 0; s4 < d; ++s4) {
                const int xc = X.colo[(size_t)i * d2 + s3 * d + s4];
                const int rc = SR.colo[(size_t)k * d + s4];
                PD_REQUIRE((xc < 0) == (rc < 0), PDMRG_ESHAPE, "merge: sector mismatch");
                if (xc < 0) continue;
                if (col0 < 0) col0 = xc - rc;
                PD_REQUIRE(xc - rc == col0, PDMRG_ESHAPE, "merge: column layout mismatch");
            }
            g.add_item(2, X.base[i] + col0, bl.dim[i], SR.cols[k], X.cols[i]);
            g.add_seg(0, SL.base[i] + lco, SL.cols[i], 1, SR.base[k], SR.cols[k], bm.dim[k]);
        }
    g.validate({SL.size, SR.size, X.size});
    g.pick_tile();
    g.finish(s);
    upload(d_rs_base, rs_base, s);
    upload(d_rs_vbase, rs_vbase, s);
    upload(d_rs_rows, rs_rows, s);
    upload(d_rs_cols, rs_cols, s);
}

void MergePlan::run(const double *psiL, const double *V, const double *psiR, double *out, double *scaled,
                    hipStream_t s) const {
    launch_row_scale(psiR, scaled, d_rs_base.as<int64_t>(), d_rs_rows.as<int32_t>(), d_rs_cols.as<int32_t>(),
                     d_rs_vbase.as<int64_t>(), (int)rs_base.size(), rs_max, V, s);
    launch_fill(out, 0.0, X.size, s);
    Slots sl{};
    sl.p[0] = psiL;
    sl.p[1] = scaled;
    sl.p[2] = out;
    g.launch(GemmPrec::F64, true, sl, s);
}

}  // namespace pdmrg
