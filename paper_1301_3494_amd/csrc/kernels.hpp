// Work-list records and kernel launchers of the pdmrg library.
//
// Every operand of a grouped launch is addressed as (slot, element offset):
// the launch passes up to kMaxSlots base pointers, so a work list built once
// for a bond stays valid for any input / output buffer of that bond.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace pdmrg {

constexpr int kMaxSlots = 8;

struct Slots {
    const void *p[kMaxSlots];
};

// One GEMM segment: C += op(A) (M x K) * op(B) (K x N); segments of an item
// share C, M, N.
struct GemmSeg {
    int64_t a_off, b_off;
    int32_t a_slot, b_slot;
    int32_t K, lda, ldb;
    int32_t pad_;
};

// C row r of an item lies at c_off + r * ldc, or, when rmap >= 0, at
// c_off + rowoff[rmap + r] (items that stack blocks of different leading
// dimensions along M).
struct GemmItem {
    int64_t c_off;
    int32_t c_slot, M, N, ldc;
    int32_t seg0, nseg;
    int32_t rmap, pad_;
};

struct GemmTile {
    int32_t item, m0, n0, pad_;
};

// A tile of a single-segment item with everything the tile needs in one
// record (the LDS-DMA kernel reads it with one scalar load); M <= 0: idle.
struct FlatTile {
    int64_t a_off, b_off, c_off;
    int32_t a_slot, b_slot, c_slot, rmap;
    int32_t M, N, K, lda, ldb, ldc, m0, n0;
};

// Scaled sum of same-shaped strided blocks: dst = sum_j coef_j * src_j.
struct LcTask {
    int64_t dst_off;
    int32_t dst_slot, rows, cols, ld;
    int32_t src0, nsrc;
};

struct LcSrc {
    int64_t off;
    int32_t slot, ld;
    double coef;
};

// Tile of a W-stage launch: elements [r0 * chunk, (r0 + 1) * chunk) of task
// `task` (row-major over its rows x cols block); chunk = c0 elements, 2048
// (8 per thread) or 512 (2 per thread, for short lists such as reductions).
constexpr int kLcChunk = 2048, kLcChunkSmall = 512;
struct LcTile {
    int32_t task, r0, c0, pad_;
};

// Rank-1 diagonal contributions of diag(H_eff): for a block of rows x cols
// (leading dim ld), out[a][b] += coef * L[a * lstride] * R[b * rstride].
struct DiagTerm {
    int64_t out_off, l_off, r_off;
    int32_t rows, cols, ld, lstride, rstride;
    int32_t pad_;
    double coef;
};

// A launch's grid size in work-items is a 32-bit count of the dispatch
// packet: blocks x threads must stay below 2^32.  Kernels over work lists
// that can be longer than that (the dot launches of a measurement at large
// bond dimension) take at most kMaxGrid workgroups and walk their tiles with
// a grid stride; check_grid throws PDMRG_ESHAPE for any launch past the limit
// (instead of a launch that fails without running).
constexpr int64_t kMaxGrid = int64_t(1) << 20;
void check_grid(int64_t blocks, int threads, const char *what);

// Frobenius product of two packed blocks of n elements: slot a at a_off and
// slot b at b_off; its value is added into output entry g.
struct DotTask {
    int64_t a_off, b_off;
    int32_t n, g;
};
// Tile of a dot launch: elements [chunk * kDotChunk, (chunk + 1) * kDotChunk)
// of task `task`.
constexpr int kDotChunk = 2048;
struct DotTile {
    int32_t task, chunk;
};

enum class GemmPrec { F64, F32, BF16X3 };

// Output tile shapes of the FP64 / FP32 kernels (4 waves, each a 32 x 32 or
// 64 x 64 sub-tile of 16 x 16 MFMA blocks); the _K16 / _K8 variants stage a
// half / quarter as much K per step (FP32 16 / 8 instead of 32, FP64 8 / 4
// instead of 16), so less LDS and more resident workgroups for short K loops.
// BF16X3 runs T64x64 only.
enum class TileShape {
    T64x64 = 0, T128x32 = 1, T32x128 = 2, T128x128 = 3,
    T64x64_K16 = 4, T128x32_K16 = 5,   // half-depth K steps
    T64x64_K8 = 6, T128x32_K8 = 7,     // quarter-depth K steps
    // FP32 / FP64, non-transposed operands: K steps of 16 staged by
    // direct-to-LDS loads (other operands: the half-depth kernel)
    T128x32_D = 8, T64x64_D = 9, T32x128_D = 10
};
constexpr int kNumShapes = 11;
constexpr unsigned kDmaShapes = (1u << 8) | (1u << 9) | (1u << 10);
inline int tile_bm(TileShape t) {
    switch (t) {
        case TileShape::T32x128: case TileShape::T32x128_D: return 32;
        case TileShape::T64x64: case TileShape::T64x64_K16: case TileShape::T64x64_K8: case TileShape::T64x64_D:
            return 64;
        default: return 128;
    }
}
inline int tile_bn(TileShape t) {
    switch (t) {
        case TileShape::T128x32: case TileShape::T128x32_K16: case TileShape::T128x32_K8: case TileShape::T128x32_D:
            return 32;
        case TileShape::T64x64: case TileShape::T64x64_K16: case TileShape::T64x64_K8: case TileShape::T64x64_D:
            return 64;
        default: return 128;
    }
}

// Launchers (defined in gemm.hip / blas.hip).  All asynchronous on `s`.
// c_is_f64: C written as double (F32 / BF16X3 inputs are float).  rowoff:
// row-offset table of the items with rmap >= 0 (may be null otherwise).
// launch_gemm: one workgroup per entry of `tiles` (in launch order; entries
// with item < 0 are idle).
void launch_gemm(GemmPrec prec, TileShape shape, bool ta, bool tb, bool c_is_f64, const Slots &slots,
                 const GemmItem *items, const GemmSeg *segs, const GemmTile *tiles, const int64_t *rowoff,
                 int ntiles, hipStream_t s);
// FP32 or FP64 operands (prec F32 / F64), non-transposed, one segment per
// item, LDS-DMA tile shape (T128x32_D, T64x64_D, T32x128_D); one workgroup per
// entry of `tiles`.
void launch_gemm_flat(GemmPrec prec, TileShape shape, bool c_is_f64, const Slots &slots, const FlatTile *tiles,
                      const int64_t *rowoff, int ntiles, hipStream_t s);
// chunk: kLcChunk or kLcChunkSmall elements per tile (as the tiles were built).
void launch_lincomb(bool f64, int chunk, const Slots &slots, const LcTask *tasks, const LcSrc *srcs,
                    const LcTile *tiles, int ntiles, hipStream_t s);
// Same with FP32 sources summed in FP32 and an FP64 destination.
// FP32 sums stored split for BF16x3 (each word a bf16 pair hi + lo, hi in the
// low half)
void launch_lincomb_split(int chunk, const Slots &slots, const LcTask *tasks, const LcSrc *srcs,
                          const LcTile *tiles, int ntiles, hipStream_t s);
void launch_lincomb_f32_f64(int chunk, const Slots &slots, const LcTask *tasks, const LcSrc *srcs,
                            const LcTile *tiles, int ntiles, hipStream_t s);
// groups[g]..groups[g+1]: the terms of output block g (all share out_off, rows,
// cols, ld); each output block is written once (zero if it has no terms).
void launch_diag_terms(const Slots &slots, const DiagTerm *terms, const int32_t *groups, int ngroups,
                       int max_rows, hipStream_t s);
// partial[t] = sum over tile t's elements of a * b (fixed-order tree).
void launch_dot_partials(const Slots &slots, int a_slot, int b_slot, const DotTask *tasks, const DotTile *tiles,
                         int ntiles, double *partial, hipStream_t s);
// out[g_of[k]] = sum over tiles t0[k]..t0[k+1] of partial (in order), for the
// k = 0..ngroups-1 output entries that have tiles.
void launch_dot_reduce(const double *partial, const int32_t *t0, const int32_t *g_of, int ngroups, double *out,
                       hipStream_t s);
void launch_convert_f64_f32(const double *x, float *y, int64_t n, hipStream_t s);
// y[i] = FP32 rounding of x[i] split into a bf16 pair (BF16x3 operands)
void launch_convert_f64_split(const double *x, uint32_t *y, int64_t n, hipStream_t s);
void launch_convert_f32_f64(const float *x, double *y, int64_t n, hipStream_t s);
void launch_fill(double *x, double v, int64_t n, hipStream_t s);
// Row scaling of row-major blocks: block k (base[k], rows[k] x cols[k]) gets
// y[r][c] = x[r][c] * scale[vbase[k] + r].
void launch_row_scale(const double *x, double *y, const int64_t *base, const int32_t *rows,
                      const int32_t *cols, const int64_t *vbase, int nblk, int max_elems,
                      const double *scale, hipStream_t s);

// Davidson helpers (FP64).
// partial[b * nvec + v] = sum over block b's range of V[v][i] * w[i]
void launch_multidot(const double *V, int64_t ldv, int nvec, const double *w, int64_t n,
                     double *partial, int nblk, hipStream_t s);
// out[v * stride] = sum_b partial[b * nvec + v] (fixed order)
void launch_reduce_partials(const double *partial, int nblk, int nvec, double *out, int stride,
                            hipStream_t s);
// y = sum_v c[v] * V[v] (+ beta * y)
void launch_combine(const double *V, int64_t ldv, int nvec, const double *c, double *y, int64_t n,
                    double beta, hipStream_t s);
// y -= sum_v c[v] * V[v]
void launch_subtract_combine(const double *V, int64_t ldv, int nvec, const double *c, double *y,
                             int64_t n, hipStream_t s);
// r = hx - theta x ; theta from dev scalar
void launch_residual(const double *hx, const double *x, const double *theta, double *r, int64_t n,
                     hipStream_t s);
// t = r / (diag - theta) with |den| >= 1e-8
void launch_precond(const double *r, const double *diag, const double *theta, double *t, int64_t n,
                    hipStream_t s);
// y = x / sqrt(*nrm2)
void launch_scale_by_inv_sqrt(const double *x, const double *nrm2, double *y, int64_t n, hipStream_t s);
// Fused Davidson passes for subspaces of at most kDavFused vectors (one read
// of every vector per pass; partial sums per block in a fixed order, reduced
// by launch_reduce_partials):
//   ritz:       x = V c, hx = HV c, r = hx - theta x, t = r / (diag - theta)
//               (|den| >= 1e-8); partial row [r.r, V_0.t, ..., V_{k-1}.t]
//   sub_dot:    t -= sum_v d[v] V[v]; partial row [V_0.t, ..., V_{k-1}.t]
//               (with_dots) or [t.t]
//   ext_gram:   partial row of w = 2 km + 1 sums (km = dav_ext_gram_width(k)):
//               V_v.HV_k at v < k, V_k.HV_k at km, HV_v.V_k at km + 1 + v
//   g_scatter:  G[v][k] and G[k][v] from that reduced row; with exact_row
//               G[0][k] = G[k][0] (the mixed-precision rule)
// Partial rows are nvec = row length apart, one per block (nblk blocks).
constexpr int kDavFused = 16;
void launch_dav_ritz(const double *V, const double *HV, int64_t ldv, int k, const double *c, const double *theta,
                     const double *diag, double *x, double *hx, double *r, double *t, int64_t n, double *partial,
                     int nblk, hipStream_t s);
void launch_dav_sub_dot(const double *V, int64_t ldv, int k, const double *d, double *t, int64_t n,
                        bool with_dots, double *partial, int nblk, hipStream_t s);
int dav_ext_gram_width(int k);
void launch_dav_ext_gram(const double *V, const double *HV, int64_t ldv, int k, int64_t n, double *partial,
                         int nblk, hipStream_t s);
void launch_dav_g_scatter(double *G, int ld, int k, const double *dots, bool exact_row, hipStream_t s);
// Lowest eigenpair of the k x k symmetric matrix G (row-major, ld) by cyclic
// Jacobi in one workgroup: theta_out[0] = eigenvalue, c_out[0..k) eigenvector
// with c[0] >= 0.
void launch_small_eig(const double *G, int k, int ld, double *theta_out, double *c_out, hipStream_t s);

// ---------------------------------------------------------------- local measurements
// Frobenius product of two column segments of one row-major block:
// sum_{r < rows, c < width} x[r * ld + ca + c] * x[r * ld + cb + c].
struct SegDot {
    const double *x;
    int32_t ld, rows, ca, cb, width, pad_;
};
// Rows [r0, r0 + kSegRows) of task `task`.
constexpr int kSegRows = 16;
struct SegTile {
    int32_t task, r0;
};
// partial[t] = tile t's share (fixed-order tree); reduce with launch_dot_reduce.
void launch_seg_dot_partials(const SegDot *tasks, const SegTile *tiles, int ntiles, double *partial, hipStream_t s);
// A square row-major block of n x n doubles.
struct SqBlock {
    double *p;
    int32_t n, pad_;
};
// Every block set to the identity.
void launch_set_identity(const SqBlock *blocks, int nblocks, int max_n, hipStream_t s);
// *out = sum over the blocks, in order, of their traces (one workgroup).
void launch_trace_sum(const SqBlock *blocks, int nblocks, double *out, hipStream_t s);

}  // namespace pdmrg
