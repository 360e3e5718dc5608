// Grouped block-sparse GEMM on CDNA4 matrix cores (gfx950).
//
// One launch runs a list of 64 x 64 output tiles drawn from many GEMM items
// (the U(1) sector blocks of one contraction, possibly of several bonds).
// Each item is C (M x N) = sum over its K-segments of op(A) op(B); the
// segments let one output block accumulate products whose operands live in
// different places (e.g. the physical-index sum of an environment update).
//
// Workgroup: 256 threads = 4 wave64, each wave owns a 32 x 32 quarter of the
// tile as 2 x 2 MFMA 16 x 16 blocks.  Operands are staged through LDS:
//   FP64 / FP32  : K-major LDS tiles, v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4;
//   BF16x3       : FP32 operands split on the fly into bf16 hi + lo halves
//                  (x = hi + lo, both rounded to nearest even), K-contiguous
//                  LDS tiles, C += hi*hi' + hi*lo' + lo*hi' with
//                  v_mfma_f32_16x16x32_bf16 and FP32 accumulation.
// Global loads of the next K-step are issued before the MFMAs of the current
// one (register double buffering).  Tiles are mapped XCD-major: the 8 XCDs
// each receive a contiguous run of the tile list, so the tiles that share an
// operand panel share an L2.
#include "kernels.hpp"

namespace pdmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned short us8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, NT = 256;

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc;
template <> struct Acc<double> { using type = d4; };
template <> struct Acc<float> { using type = f4; };

__device__ __forceinline__ int map_tile(int ntiles) {
    const int chunk = (ntiles + 7) / 8;
    return (blockIdx.x % 8) * chunk + blockIdx.x / 8;
}

// Iterates the (segment, k0) steps of one item.
struct KIter {
    int seg, k0, nseg;
};

// ---------------------------------------------------------------- FP64 / FP32
template <typename T, typename TC, bool TA, bool TB>
__global__ __launch_bounds__(NT) void gemm_kmajor(Slots slots, const GemmItem *__restrict__ items,
                                                  const GemmSeg *__restrict__ segs,
                                                  const GemmTile *__restrict__ tiles, int ntiles) {
    constexpr int BK = 16;
    const int t = map_tile(ntiles);
    if (t >= ntiles) return;
    const GemmTile tile = tiles[t];
    const GemmItem it = items[tile.item];
    __shared__ T As[BK][BM + 2];
    __shared__ T Bs[BK][BN + 2];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int m0 = tile.m0, n0 = tile.n0;
    using V4 = typename Acc<T>::type;
    V4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = V4{0, 0, 0, 0};

    // thread -> load coordinates (4 elements of A and of B per K-step)
    const int a_r = TA ? (tid & 15) * 4 : tid >> 2;   // m (first of 4 if TA)
    const int a_k = TA ? tid >> 4 : (tid & 3) * 4;    // k (first of 4 if !TA)
    const int b_n = TB ? tid >> 2 : (tid & 15) * 4;
    const int b_k = TB ? (tid & 3) * 4 : tid >> 4;

    T ra[4], rb[4];
    auto load = [&](const GemmSeg &sg, int k0) {
        const T *A = static_cast<const T *>(slots.p[sg.a_slot]) + sg.a_off;
        const T *B = static_cast<const T *>(slots.p[sg.b_slot]) + sg.b_off;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int gm = m0 + a_r + (TA ? u : 0), gk = k0 + a_k + (TA ? 0 : u);
            ra[u] = (gm < it.M && gk < sg.K)
                        ? (TA ? A[(int64_t)gk * sg.lda + gm] : A[(int64_t)gm * sg.lda + gk])
                        : T(0);
            const int gn = n0 + b_n + (TB ? 0 : u), gkb = k0 + b_k + (TB ? u : 0);
            rb[u] = (gn < it.N && gkb < sg.K)
                        ? (TB ? B[(int64_t)gn * sg.ldb + gkb] : B[(int64_t)gkb * sg.ldb + gn])
                        : T(0);
        }
    };

    int sidx = 0, k0 = 0;
    // skip empty segments
    while (sidx < it.nseg && segs[it.seg0 + sidx].K <= 0) ++sidx;
    GemmSeg sg;
    if (sidx < it.nseg) {
        sg = segs[it.seg0 + sidx];
        load(sg, 0);
    }
    while (sidx < it.nseg) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (TA) As[a_k][a_r + u] = ra[u]; else As[a_k + u][a_r] = ra[u];
            if (TB) Bs[b_k + u][b_n] = rb[u]; else Bs[b_k][b_n + u] = rb[u];
        }
        __syncthreads();
        // advance and prefetch the next step
        k0 += BK;
        if (k0 >= sg.K) {
            k0 = 0;
            ++sidx;
            while (sidx < it.nseg && segs[it.seg0 + sidx].K <= 0) ++sidx;
            if (sidx < it.nseg) sg = segs[it.seg0 + sidx];
        }
        if (sidx < it.nseg) load(sg, k0);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4), c = lane & 15;
            const T a0 = As[kr][wm + c], a1 = As[kr][wm + 16 + c];
            const T b0 = Bs[kr][wn + c], b1 = Bs[kr][wn + 16 + c];
            acc[0][0] = mfma16(a0, b0, acc[0][0]);
            acc[0][1] = mfma16(a0, b1, acc[0][1]);
            acc[1][0] = mfma16(a1, b0, acc[1][0]);
            acc[1][1] = mfma16(a1, b1, acc[1][1]);
        }
    }
    // Result rows held by (lane, register r): v_mfma_f64_16x16x4 returns row
    // 4 r + lane/16, v_mfma_f32_16x16x4 row 4 (lane/16) + r; column lane % 16.
    constexpr bool kF64 = sizeof(T) == 8;
    TC *C = static_cast<TC *>(const_cast<void *>(slots.p[it.c_slot])) + it.c_off;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = kF64 ? r * 4 + (lane >> 4) : (lane >> 4) * 4 + r;
                const int gm = m0 + wm + i * 16 + row;
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm < it.M && gn < it.N) C[(int64_t)gm * it.ldc + gn] = (TC)acc[i][j][r];
            }
}

// ---------------------------------------------------------------- BF16 x3
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    // bfloat16 = upper 16 bits of binary32, rounded to nearest even
    unsigned int u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
    return __uint_as_float(((unsigned int)h) << 16);
}

template <typename TC, bool TA, bool TB>
__global__ __launch_bounds__(NT) void gemm_bf16x3(Slots slots, const GemmItem *__restrict__ items,
                                                  const GemmSeg *__restrict__ segs,
                                                  const GemmTile *__restrict__ tiles, int ntiles) {
    constexpr int BK = 32, LD = BK + 8;   // 80-byte LDS rows keep 16-byte alignment
    const int t = map_tile(ntiles);
    if (t >= ntiles) return;
    const GemmTile tile = tiles[t];
    const GemmItem it = items[tile.item];
    __shared__ __attribute__((aligned(16))) unsigned short Ah[BM][LD], Al[BM][LD];
    __shared__ __attribute__((aligned(16))) unsigned short Bh[BN][LD], Bl[BN][LD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int m0 = tile.m0, n0 = tile.n0;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0, 0, 0, 0};

    // 8 elements of A and of B per thread and K-step
    const int a_r = TA ? (tid & 7) * 8 : tid >> 2;
    const int a_k = TA ? tid >> 3 : (tid & 3) * 8;
    const int b_n = TB ? tid >> 2 : (tid & 7) * 8;
    const int b_k = TB ? (tid & 3) * 8 : tid >> 3;

    float ra[8], rb[8];
    auto load = [&](const GemmSeg &sg, int k0) {
        const float *A = static_cast<const float *>(slots.p[sg.a_slot]) + sg.a_off;
        const float *B = static_cast<const float *>(slots.p[sg.b_slot]) + sg.b_off;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int gm = m0 + a_r + (TA ? u : 0), gk = k0 + a_k + (TA ? 0 : u);
            ra[u] = (gm < it.M && gk < sg.K)
                        ? (TA ? A[(int64_t)gk * sg.lda + gm] : A[(int64_t)gm * sg.lda + gk])
                        : 0.f;
            const int gn = n0 + b_n + (TB ? 0 : u), gkb = k0 + b_k + (TB ? u : 0);
            rb[u] = (gn < it.N && gkb < sg.K)
                        ? (TB ? B[(int64_t)gn * sg.ldb + gkb] : B[(int64_t)gkb * sg.ldb + gn])
                        : 0.f;
        }
    };

    int sidx = 0, k0 = 0;
    while (sidx < it.nseg && segs[it.seg0 + sidx].K <= 0) ++sidx;
    GemmSeg sg;
    if (sidx < it.nseg) {
        sg = segs[it.seg0 + sidx];
        load(sg, 0);
    }
    while (sidx < it.nseg) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const unsigned short ha = bf16_rne(ra[u]);
            const unsigned short la = bf16_rne(ra[u] - bf16_to_f32(ha));
            const unsigned short hb = bf16_rne(rb[u]);
            const unsigned short lb = bf16_rne(rb[u] - bf16_to_f32(hb));
            if (TA) { Ah[a_r + u][a_k] = ha; Al[a_r + u][a_k] = la; }
            else    { Ah[a_r][a_k + u] = ha; Al[a_r][a_k + u] = la; }
            if (TB) { Bh[b_n][b_k + u] = hb; Bl[b_n][b_k + u] = lb; }
            else    { Bh[b_n + u][b_k] = hb; Bl[b_n + u][b_k] = lb; }
        }
        __syncthreads();
        k0 += BK;
        if (k0 >= sg.K) {
            k0 = 0;
            ++sidx;
            while (sidx < it.nseg && segs[it.seg0 + sidx].K <= 0) ++sidx;
            if (sidx < it.nseg) sg = segs[it.seg0 + sidx];
        }
        if (sidx < it.nseg) load(sg, k0);
        const int r = lane & 15, kq = (lane >> 4) * 8;
        bf8 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            ah[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(&Ah[wm + i * 16 + r][kq]));
            al[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(&Al[wm + i * 16 + r][kq]));
            bh[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(&Bh[wn + i * 16 + r][kq]));
            bl[i] = __builtin_bit_cast(bf8, *reinterpret_cast<const us8 *>(&Bl[wn + i * 16 + r][kq]));
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
            }
    }
    TC *C = static_cast<TC *>(const_cast<void *>(slots.p[it.c_slot])) + it.c_off;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gm < it.M && gn < it.N) C[(int64_t)gm * it.ldc + gn] = (TC)acc[i][j][r];
            }
}

// ---------------------------------------------------------------- launcher
template <typename T, typename TC>
static void dispatch_kmajor(bool ta, bool tb, dim3 g, hipStream_t s, const Slots &sl,
                            const GemmItem *it, const GemmSeg *sg, const GemmTile *tl, int n) {
    if (!ta && !tb) hipLaunchKernelGGL((gemm_kmajor<T, TC, false, false>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
    else if (ta && !tb) hipLaunchKernelGGL((gemm_kmajor<T, TC, true, false>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
    else if (!ta && tb) hipLaunchKernelGGL((gemm_kmajor<T, TC, false, true>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
    else hipLaunchKernelGGL((gemm_kmajor<T, TC, true, true>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
}

template <typename TC>
static void dispatch_bf16(bool ta, bool tb, dim3 g, hipStream_t s, const Slots &sl,
                          const GemmItem *it, const GemmSeg *sg, const GemmTile *tl, int n) {
    if (!ta && !tb) hipLaunchKernelGGL((gemm_bf16x3<TC, false, false>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
    else if (ta && !tb) hipLaunchKernelGGL((gemm_bf16x3<TC, true, false>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
    else if (!ta && tb) hipLaunchKernelGGL((gemm_bf16x3<TC, false, true>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
    else hipLaunchKernelGGL((gemm_bf16x3<TC, true, true>), g, dim3(NT), 0, s, sl, it, sg, tl, n);
}

void launch_gemm(GemmPrec prec, bool ta, bool tb, bool c_is_f64, const Slots &slots,
                 const GemmItem *items, const GemmSeg *segs, const GemmTile *tiles, int ntiles,
                 hipStream_t s) {
    if (ntiles <= 0) return;
    const int chunk = (ntiles + 7) / 8;
    dim3 grid(chunk * 8);
    switch (prec) {
        case GemmPrec::F64:
            dispatch_kmajor<double, double>(ta, tb, grid, s, slots, items, segs, tiles, ntiles);
            break;
        case GemmPrec::F32:
            if (c_is_f64) dispatch_kmajor<float, double>(ta, tb, grid, s, slots, items, segs, tiles, ntiles);
            else dispatch_kmajor<float, float>(ta, tb, grid, s, slots, items, segs, tiles, ntiles);
            break;
        case GemmPrec::BF16X3:
            if (c_is_f64) dispatch_bf16<double>(ta, tb, grid, s, slots, items, segs, tiles, ntiles);
            else dispatch_bf16<float>(ta, tb, grid, s, slots, items, segs, tiles, ntiles);
            break;
    }
}

}  // namespace pdmrg
