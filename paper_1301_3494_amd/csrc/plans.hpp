// Contraction plans: host-built work lists of the grouped GEMM and W-stage
// launches for H_eff, environment updates and the merge.
#pragma once
#include "common.hpp"
#include "kernels.hpp"

namespace pdmrg {

struct LcList;

// Rows [r0, r0 + rows) of a stacked item: C row r0 + r lies at c_off + r * ldc.
struct RowBlock {
    int64_t c_off;
    int32_t r0, rows, ldc;
};

// Device copies of a list's records (tiles in launch order).
struct GemmDev {
    const GemmItem *items;
    const GemmSeg *segs;
    const GemmTile *tiles;
    const FlatTile *ftiles;
    const int64_t *rowoff;
};
struct LcDev {
    const LcTask *tasks;
    const LcSrc *srcs;
    const LcTile *tiles;
};

struct GemmList {
    bool ta = false, tb = false;
    int elem_bytes = 8;                    // operand element size (4 in the FP32 / BF16x3 modes)
    TileShape shape = TileShape::T64x64;   // set by pick_tile()
    unsigned shapes_allowed = ((1u << kNumShapes) - 1) & ~kDmaShapes;   // H_eff plans add kDmaShapes
    std::vector<GemmItem> items;
    std::vector<GemmSeg> segs;
    std::vector<GemmTile> tiles;           // in launch order (workgroup b runs tiles[b]); item < 0: idle
    int ntiles_real = 0;                   // tiles that compute (without the idle padding)
    std::vector<int64_t> rowoff;           // row offsets of stacked items
    std::vector<int32_t> blk0;             // per item: first RowBlock, -1 for a plain item
    std::vector<RowBlock> blocks;
    double flops = 0.0;
    DevBuf d_items, d_segs, d_tiles, d_rowoff;
    // LDS-DMA shapes on lists of single-segment items: the tiles as FlatTile
    // records in the same launch order (used by launch() for FP32 and FP64)
    std::vector<FlatTile> ftiles;
    DevBuf d_ftiles;

    int add_item(int c_slot, int64_t c_off, int M, int N, int ldc);
    // An item whose M rows stack the given output blocks (each N wide).
    int add_stacked_item(int c_slot, int N, const std::vector<RowBlock> &blks);
    void add_seg(int a_slot, int64_t a_off, int lda, int b_slot, int64_t b_off, int ldb, int K);
    // Tile shape of least estimated time: padded MFMA work over the fraction of
    // the device that the tiles (times the split-K factor they allow) can fill.
    void pick_tile();
    int ntiles_for(TileShape t) const;
    double padded_flops(TileShape t) const;
    // Build the tiles and place them for the launch (see place_tiles), upload.
    void finish(hipStream_t s);
    // The host part of finish: tiles (and flat tiles) in launch order.
    void build_tiles();
    void launch(GemmPrec prec, bool c_is_f64, const Slots &sl, hipStream_t s) const;
    // Same with the records at caller-provided device addresses.
    void launch(GemmPrec prec, bool c_is_f64, const Slots &sl, const GemmDev &dv, hipStream_t s) const;
    // Copy of the host-side lists (no device buffers).
    GemmList host_copy() const;
    // Throws unless every element an item touches lies inside its slot's
    // buffer (sizes in elements, per slot).
    void validate(const std::vector<int64_t> &slot_elems) const;
    // Split-K: the item of longest K is cut into `parts` items over
    // consecutive K ranges and every other item into as many as keep its
    // ranges near the same length (at most 8, at least 1), each writing a
    // partial product into slot
    // `pslot` (packed, ld = N); `reduce` receives one task per original item
    // that sums its partials into the original C in a fixed order.  Returns
    // the number of partial elements.  Call before validate / finish.
    // all = true: items too short to split are still written as one part, so
    // the whole list writes slot `pslot` (e.g. partials of another precision).
    int64_t split_k(int parts, int pslot, LcList &reduce, bool all = false);
};

struct LcList {
    int chunk = kLcChunk;   // elements per tile (kLcChunkSmall for short lists)
    std::vector<LcTask> tasks;
    std::vector<LcSrc> srcs;
    std::vector<LcTile> tiles;
    double flops = 0.0;
    int64_t elems_out = 0, elems_in = 0;
    DevBuf d_tasks, d_srcs, d_tiles;

    int add_task(int dst_slot, int64_t dst_off, int rows, int cols, int ld);
    void add_src(int slot, int64_t off, int ld, double coef);
    void finish(hipStream_t s);
    void build_tiles();   // the host part of finish
    void launch(bool f64, const Slots &sl, hipStream_t s) const;
    void launch(bool f64, const Slots &sl, const LcDev &dv, hipStream_t s) const;
    void launch_f32_to_f64(const Slots &sl, hipStream_t s) const;
    // FP32 sums written as split bf16 pairs (BF16x3 operands)
    void launch_split(const Slots &sl, hipStream_t s) const;
    void validate(const std::vector<int64_t> &slot_elems) const;
};

// y = H_eff x on bonds (bl, br) -- stage 1: T1 = L x (per ket sector, the
// MPO channels stacked on M); stage 2: T2 = (W1 W2) T1 (W stage); stage 3:
// y = T2 R (per output block, the (channel, ket) pairs stacked on K), split
// along K when its output tiles alone cannot fill the device.
struct HeffPlan {
    Bond bl, br;
    Phys p;
    SiteLayout X;
    EnvLayout Lt, Rt;
    int64_t nT1 = 0, nT2 = 0, nP = 0;
    GemmList g1, g3;
    GemmList g3_base;   // stage 3 before split-K
    // W stage; split-K reduction of stage 3 (partials in slot 6: FP64 in FP64
    // mode; FP32 for every item in the FP32 / BF16x3 modes)
    LcList w, r3;
    bool lowp = false;
    int parts3 = 1;
    // Re-tile stage 1 / stage 3 (stage 3 is re-split: parts <= 0 picks the
    // K split that gives >= 1024 tiles).
    void set_g1_shape(TileShape t, hipStream_t s);
    void set_g3_shape(TileShape t, hipStream_t s, int parts = 0);
    int default_parts(TileShape t) const;
    std::vector<DiagTerm> diag_terms;
    std::vector<int32_t> diag_groups;
    int diag_max_rows = 0;
    void build(const Bond &bl_, const Bond &br_, const Phys &p_, const MpoSite &W1, const MpoSite &W2,
               int prec, hipStream_t s);
};

// Environment updates (dir +1: L on bl -> L on br; dir -1: R on br -> R on bl).
struct EnvPlan {
    int dir = 1;
    Bond bl, br;
    Phys p;
    SiteLayout S;
    EnvLayout Ein, Eout, Aux;
    int64_t nU1 = 0, nU2 = 0;
    GemmList g1, g3;
    LcList w;
    // upload = false: host work lists only (counts, no device buffers).
    void build(int dir_, const Bond &bl_, const Bond &br_, const Phys &p_, const MpoSite &W, hipStream_t s,
               bool upload = true);
    // slots: 0 env_in, 1 site, 2 env_out, 3 U1, 4 U2
    void run(GemmPrec prec, const void *env_in, const void *site, void *env_out, void *U1, void *U2,
             hipStream_t s) const;
    // Same with the work-list records at caller-provided device addresses
    // (plan built with upload = false and the lists' build_tiles() called).
    void run(GemmPrec prec, const void *env_in, const void *site, void *env_out, void *U1, void *U2,
             const GemmDev &d1, const LcDev &dw, const GemmDev &d3, hipStream_t s) const;
};

// Psi' = psiL V psiR (Eq. eqn:merge).
struct MergePlan {
    Bond bl, bm, br;
    Phys p;
    SiteLayout SL, SR, X;
    GemmList g;
    std::vector<int64_t> rs_base, rs_vbase;
    std::vector<int32_t> rs_rows, rs_cols;
    DevBuf d_rs_base, d_rs_vbase, d_rs_rows, d_rs_cols;
    int rs_max = 0;
    void build(const Bond &bl_, const Bond &bm_, const Bond &br_, const Phys &p_, hipStream_t s);
    void run(const double *psiL, const double *V, const double *psiR, double *out, double *scaled,
             hipStream_t s) const;
};

// Gradient of <psi|H|psi> with respect to one MPO tensor W[w, s, t, w'] at a
// single-site centre psi on (bl, br):
//   G[w, s, t, w'] = sum L[a, w, a'] psi[a, s, b] psi[a', t, b'] R[b, w', b'].
// Stage 1: U1[j] = Lket[j] psi[j] (rows (w, a), cols (t, b')) -- the first
// stage of an environment update.  Stage 2: per (a sector, w, s, t) the block
// Z = U1[(w, a), (t, b')]^T psi[a, (s, b)] over a, laid out [b'][b] like the
// R blocks.  Stage 3: G entries as Frobenius products <Z, R[w']> over the
// channels w' whose charge matches, summed in a fixed order.
struct GradPlan {
    Bond bl, br;
    Phys p;
    int Dl = 0, Dr = 0;
    SiteLayout S;
    EnvLayout Lt, Rt;
    int64_t nU1 = 0, nZ = 0;
    GemmList g1, gz;
    std::vector<DotTask> dots;
    std::vector<DotTile> dtiles;
    std::vector<int32_t> t0, g_of;   // tiles of output entry g_of[k]: t0[k] .. t0[k+1]
    DevBuf d_dots, d_dtiles, d_t0, d_gof;
    double flops = 0.0;
    void build(const Bond &bl_, const Bond &br_, const Phys &p_, const MpoSite &W, hipStream_t s);
    // slots: 0 L, 1 psi, 2 R, 3 U1, 4 Z; partial holds dtiles.size() doubles;
    // G (Dl d d Dr) is overwritten.
    void run(const double *L, const double *psi, const double *R, double *U1, double *Z, double *partial,
             double *G, hipStream_t s) const;
};

std::vector<double> two_site_mpo(const MpoSite &W1, const MpoSite &W2);

}  // namespace pdmrg
