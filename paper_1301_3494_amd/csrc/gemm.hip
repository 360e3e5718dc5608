// Grouped block-sparse GEMM on CDNA4 matrix cores (gfx950).
//
// One launch runs a list of output tiles drawn from many GEMM items (the U(1)
// sector blocks of one contraction, possibly of several bonds).  Each item is
// C (M x N) = sum over its K-segments of op(A) op(B); the segments let one
// output block accumulate products whose operands live in different places
// (e.g. the physical-index sum of an environment update).  An item may stack
// blocks with different output leading dimensions along M through a row
// offset table.
//
// Workgroup: 256 threads = 4 wave64.  FP64 / FP32 tiles are BM x BN with the
// waves on a WGM x WGN grid, each wave owning an (BM/WGM) x (BN/WGN) sub-tile
// of 16 x 16 MFMA blocks (v_mfma_f64_16x16x4 / v_mfma_f32_16x16x4).  BF16x3
// takes operands split once in memory (each 4-byte word a bf16 pair x = hi +
// lo, both rounded to nearest even) through the FP32 LDS-DMA pipeline and
// accumulates lo*hi' + hi*lo' + hi*hi' with v_mfma_f32_16x16x16_bf16 in FP32.
//
// Operands are read with buffer loads: the descriptor of each segment spans
// its operand and an offset outside it returns zero, so ragged tile edges need
// no branches.  Global loads of the next K-step are issued before the MFMAs of
// the current one.  Workgroup b runs tiles[b]: the host places the tiles so
// that every XCD (b % 8) receives an even share of the work and the tiles
// that share an A panel share one XCD's L2.
#include "kernels.hpp"

namespace pdmrg {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NT = 256;

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T> struct Acc;
template <> struct Acc<double> { using type = d4; };
template <> struct Acc<float> { using type = f4; };

// A pointer that is the same in every lane, held in scalar registers.
__device__ __forceinline__ void *uniform_ptr(const void *p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
}

// Raw buffer descriptor over [p, p + 2 GiB): an offset at or beyond kOutOfRange
// reads as zero.
constexpr unsigned kOutOfRange = 0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t operand_rsrc(const void *p) {
    return __builtin_amdgcn_make_buffer_rsrc(uniform_ptr(p), 0, 0x7fffffff, 0x00020000);
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Element offset of row r of an item's C.
__device__ __forceinline__ int64_t c_row(const GemmItem &it, const int64_t *__restrict__ rowoff, int r) {
    return it.rmap >= 0 ? rowoff[it.rmap + r] : (int64_t)r * it.ldc;
}

// ---------------------------------------------------------------- FP64 / FP32
// LDS tiles are M-major (A) / N-major (B) with the K index contiguous and an
// odd row stride (BK + 1 elements), so the global->LDS stores of either
// operand orientation and the MFMA operand reads (16 lanes = 16 rows, same k)
// spread over the banks.  Two LDS buffers: the next K-step's global loads are
// in flight during the current MFMAs and one barrier separates steps.
template <typename T> struct KStep;
template <> struct KStep<double> { static constexpr int BK = 16; };
template <> struct KStep<float> { static constexpr int BK = 32; };

// KDIV = 2 / 4: a half / quarter of the K step (and LDS) of KStep.
template <typename T, typename TC, bool TA, bool TB, int BM, int BN, int WGM, int KDIV>
__global__ __launch_bounds__(NT) void gemm_kmajor(Slots slots, const GemmItem *__restrict__ items,
                                                  const GemmSeg *__restrict__ segs,
                                                  const GemmTile *__restrict__ tiles,
                                                  const int64_t *__restrict__ rowoff, int ntiles) {
    constexpr int WGN = 4 / WGM;
    constexpr int BK = KStep<T>::BK / KDIV, LDK = BK + 1;
    constexpr int NLA = BM * BK / NT, NLB = BN * BK / NT;   // elements per thread and step
    constexpr int SM = BM / WGM, SN = BN / WGN;              // wave sub-tile
    constexpr int WBM = SM / 16, WBN = SN / 16;              // MFMA blocks per wave
    static_assert(NT % BK == 0 && NT % BM == 0 && NT % BN == 0 && WBM >= 1 && WBN >= 1, "tile shape");
    // the host has placed the tiles in launch order (idle tiles: item < 0)
    if ((int)blockIdx.x >= ntiles) return;
    const GemmTile tile = tiles[blockIdx.x];
    if (tile.item < 0) return;
    const GemmItem it = items[tile.item];
    __shared__ T As[2][BM][LDK];
    __shared__ T Bs[2][BN][LDK];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = (wave / WGN) * SM, wn = (wave % WGN) * SN;
    const int m0 = tile.m0, n0 = tile.n0;
    using V4 = typename Acc<T>::type;
    V4 acc[WBM][WBN];
#pragma unroll
    for (int i = 0; i < WBM; ++i)
#pragma unroll
        for (int j = 0; j < WBN; ++j) acc[i][j] = V4{0, 0, 0, 0};

    // coalesced thread -> element maps: consecutive threads walk the
    // contiguous global index of each operand
    //   A (M x K):  K contiguous (!TA): k = tid % BK, m = tid / BK + u * (NT / BK)
    //               M contiguous (TA):  m = tid % BM, k = tid / BM + u * (NT / BM)
    //   B (K x N):  N contiguous (!TB): n = tid % BN, k = tid / BN + u * (NT / BN)
    //               K contiguous (TB):  k = tid % BK, n = tid / BK + u * (NT / BK)
    auto a_idx = [&](int u, int &m, int &k) {
        if (TA) { m = tid % BM; k = tid / BM + u * (NT / BM); }
        else    { k = tid % BK; m = tid / BK + u * (NT / BK); }
    };
    auto b_idx = [&](int u, int &n, int &k) {
        if (TB) { k = tid % BK; n = tid / BK + u * (NT / BK); }
        else    { n = tid % BN; k = tid / BN + u * (NT / BN); }
    };
    T ra[NLA], rb[NLB];
    int K = 0, lda = 0, ldb = 0;
    __amdgpu_buffer_rsrc_t rA, rB;
    auto set_seg = [&](const GemmSeg &sg) {
        K = __builtin_amdgcn_readfirstlane(sg.K);
        lda = __builtin_amdgcn_readfirstlane(sg.lda);
        ldb = __builtin_amdgcn_readfirstlane(sg.ldb);
        rA = operand_rsrc(static_cast<const T *>(slots.p[sg.a_slot]) + sg.a_off);
        rB = operand_rsrc(static_cast<const T *>(slots.p[sg.b_slot]) + sg.b_off);
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int u = 0; u < NLA; ++u) {
            int m, k;
            a_idx(u, m, k);
            const int gm = m0 + m, gk = k0 + k;
            const unsigned off = TA ? (unsigned)(gk * lda + gm) : (unsigned)(gm * lda + gk);
            ra[u] = buf_load(rA, (gm < it.M && gk < K) ? off * (unsigned)sizeof(T) : kOutOfRange, T());
        }
#pragma unroll
        for (int u = 0; u < NLB; ++u) {
            int n, k;
            b_idx(u, n, k);
            const int gn = n0 + n, gk = k0 + k;
            const unsigned off = TB ? (unsigned)(gn * ldb + gk) : (unsigned)(gk * ldb + gn);
            rb[u] = buf_load(rB, (gn < it.N && gk < K) ? off * (unsigned)sizeof(T) : kOutOfRange, T());
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int u = 0; u < NLA; ++u) {
            int m, k;
            a_idx(u, m, k);
            As[buf][m][k] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < NLB; ++u) {
            int n, k;
            b_idx(u, n, k);
            Bs[buf][n][k] = rb[u];
        }
    };

    int sidx = 0, k0 = 0;
    while (sidx < it.nseg && segs[it.seg0 + sidx].K <= 0) ++sidx;
    int buf = 0;
    if (sidx < it.nseg) {
        set_seg(segs[it.seg0 + sidx]);
        load(0);
        store(0);
    }
    __syncthreads();
    while (sidx < it.nseg) {
        // advance to the next step and prefetch it
        k0 += BK;
        if (k0 >= K) {
            k0 = 0;
            ++sidx;
            while (sidx < it.nseg && segs[it.seg0 + sidx].K <= 0) ++sidx;
            if (sidx < it.nseg) set_seg(segs[it.seg0 + sidx]);
        }
        const bool more = sidx < it.nseg;
        if (more) load(k0);
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const int kr = kk + (lane >> 4), c = lane & 15;
            T a[WBM], b[WBN];
#pragma unroll
            for (int i = 0; i < WBM; ++i) a[i] = As[buf][wm + i * 16 + c][kr];
#pragma unroll
            for (int j = 0; j < WBN; ++j) b[j] = Bs[buf][wn + j * 16 + c][kr];
#pragma unroll
            for (int i = 0; i < WBM; ++i)
#pragma unroll
                for (int j = 0; j < WBN; ++j) acc[i][j] = mfma16(a[i], b[j], acc[i][j]);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // Result rows held by (lane, register r): v_mfma_f64_16x16x4 returns row
    // 4 r + lane/16, v_mfma_f32_16x16x4 row 4 (lane/16) + r; column lane % 16.
    constexpr bool kF64 = sizeof(T) == 8;
    TC *C = static_cast<TC *>(const_cast<void *>(slots.p[it.c_slot])) + it.c_off;
#pragma unroll
    for (int i = 0; i < WBM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = kF64 ? r * 4 + (lane >> 4) : (lane >> 4) * 4 + r;
            const int gm = m0 + wm + i * 16 + row;
            if (gm >= it.M) continue;
            TC *Cr = C + c_row(it, rowoff, gm);
#pragma unroll
            for (int j = 0; j < WBN; ++j) {
                const int gn = n0 + wn + j * 16 + (lane & 15);
                if (gn < it.N) Cr[gn] = (TC)acc[i][j][r];
            }
        }
}

// ---------------------------------------------------------------- LDS DMA
// Non-transposed FP32 / FP64 operands (A: K contiguous, B: N contiguous) staged by
// buffer loads that write LDS directly (no register staging), NS stages deep:
// the loads of the next NS - 1 K-steps are in flight while the MFMAs of the
// current one run, and one barrier separates steps.  Each load instruction
// writes 64 consecutive dwords (lane i -> dword i), so the LDS layout follows
// from which element each lane fetches:
//   A stage: groups of 4 FP32 (2 FP64) rows x 16 k (64 dwords, one
//     instruction, whole 64-byte (128-byte) row pieces from global memory),
//     consecutive groups 68 dwords apart;
//   B stage: the 16 x BN tile row-major in 64-dword chunks (one instruction
//     each, whole row pieces), FP32 chunks 64 + 256 / BN dwords apart, FP64
//     chunks unpadded.
// Within a K-step, lane group g (lane / 16) of MFMA s (0..3) takes k = 4 g + s
// (the same permutation of k for A and B, so the sum is unchanged): a lane's
// four A values are adjacent (one 16-byte LDS read in FP32, two in FP64), and
// with the layouts above every LDS read of the MFMA operands touches each
// bank once per cycle (FP32 B reads serve 32 lanes a cycle, across k rows,
// hence the padding; FP64 B reads serve 16 lanes, one k row).
// The loads are written in inline assembly because the compiler, which tracks
// LDS written by its own direct loads, waits for all of them before any LDS
// read and so would drain the pipeline at every step; these loads have no
// register results, and the stage waits below are explicit.  A tile arrives
// as one FlatTile record (one scalar load): with several workgroups starting
// together on a CU, a chain of dependent descriptor loads (tile, item,
// segment) left the CU idle for microseconds at every tile start.
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ u32x4 dma_rsrc(const void *p) {
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    u32x4 r;
    r.x = __builtin_amdgcn_readfirstlane((uint32_t)a);
    r.y = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32)) & 0xffffu;
    r.z = 0x7fffffffu;   // 2 GiB range: offsets >= kOutOfRange read zero
    r.w = 0x00020000u;   // 32-bit data format
    return r;
}

#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Winline-asm"
// LDS[lds + 4 lane] = dword at byte offset voff of the buffer (0 if out of range)
__device__ __forceinline__ void dma_dword(u32x4 rsrc, uint32_t lds, uint32_t voff) {
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dword %1, %2, 0 offen lds"
                 :: "s"(lds), "v"(voff), "s"(rsrc) : "memory", "m0");
}
#pragma clang diagnostic pop

template <int N> __device__ __forceinline__ void wait_vm() {
    asm volatile("s_waitcnt vmcnt(%0)" :: "n"(N) : "memory");
}

// SPLIT (BF16x3): every 4-byte operand word holds a value as two bf16, the
// high part in its low half and the low part in its high half (x = hi + lo);
// the staging is the FP32 kernel's, and each K step of 16 issues three
// v_mfma_f32_16x16x16_bf16 (lo * hi', hi * lo', hi * hi', small terms first)
// in place of four v_mfma_f32_16x16x4_f32.
typedef __bf16 bf2 __attribute__((ext_vector_type(2)));
typedef short s4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s4v split_hi(float w0, float w1, float w2, float w3) {
    const unsigned a = __builtin_bit_cast(unsigned, w0), b = __builtin_bit_cast(unsigned, w1);
    const unsigned c = __builtin_bit_cast(unsigned, w2), d = __builtin_bit_cast(unsigned, w3);
    return __builtin_bit_cast(s4v, u2v{(a & 0xffffu) | (b << 16), (c & 0xffffu) | (d << 16)});
}
__device__ __forceinline__ s4v split_lo(float w0, float w1, float w2, float w3) {
    const unsigned a = __builtin_bit_cast(unsigned, w0), b = __builtin_bit_cast(unsigned, w1);
    const unsigned c = __builtin_bit_cast(unsigned, w2), d = __builtin_bit_cast(unsigned, w3);
    return __builtin_bit_cast(s4v, u2v{(a >> 16) | (b & 0xffff0000u), (c >> 16) | (d & 0xffff0000u)});
}

template <typename T, typename TC, int BM, int BN, int WGM, int NS, bool SPLIT = false>
__global__ __launch_bounds__(NT) void gemm_dma(Slots slots, const FlatTile *__restrict__ tiles,
                                               const int64_t *__restrict__ rowoff, int ntiles) {
    constexpr int BK = 16;
    constexpr int EW = sizeof(T) / 4;                            // dwords per element
    constexpr int RG = 4 / EW;                                   // rows per A load group (64 dwords)
    constexpr int WGN = 4 / WGM;
    constexpr int SM = BM / WGM, SN = BN / WGN;
    constexpr int WBM = SM / 16, WBN = SN / 16;
    constexpr int AGS = 68, A_DW = (BM / RG) * AGS;              // A: groups of RG rows
    // B: 64-dword chunks of the row-major 16 x BN tile; FP32 reads (32 lanes a
    // cycle, four k rows) need the padding, FP64 reads (16 lanes) do not
    constexpr int PB = EW == 1 ? 256 / BN : 0, BCS = 64 + PB, B_DW = (BK * BN * EW / 64) * BCS;
    constexpr int ST_DW = A_DW + B_DW;                           // one stage, dwords
    constexpr int NA = BM / RG / 4, NB = BK * BN * EW / 256;     // loads per wave and step
    constexpr int NL = NA + NB;
    static_assert(NS >= 2 && NS <= 4 && WBM >= 1 && WBN >= 1 && BN <= 128 && NA >= 1 && NB >= 1 &&
                  (NS - 2) * NL <= 63, "shape");
    static_assert(A_DW % 4 == 0 && ST_DW % 4 == 0, "16-byte aligned A reads");
    using V4 = typename Acc<T>::type;
    __shared__ __attribute__((aligned(16))) float sm[NS * ST_DW];

    if ((int)blockIdx.x >= ntiles) return;
    const FlatTile ft = tiles[blockIdx.x];
    if (ft.M <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = (wave / WGN) * SM, wn = (wave % WGN) * SN;
    const int M = ft.M, N = ft.N, K = ft.K, m0 = ft.m0, n0 = ft.n0;
    const uint32_t lds0 = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) float *)sm;
    const u32x4 rA = dma_rsrc(static_cast<const T *>(slots.p[ft.a_slot]) + ft.a_off);
    const u32x4 rB = dma_rsrc(static_cast<const T *>(slots.p[ft.b_slot]) + ft.b_off);
    const int nsteps = K > 0 ? (K + BK - 1) / BK : 0;

    // A load: lane -> row a_r of the group, element a_k of the 16, dword a_h of it
    const int a_r = lane / (16 * EW), a_k = (lane % (16 * EW)) / EW, a_h = lane % EW;
    // per-lane byte offsets of this lane's A rows and B columns (out of range: kOutOfRange)
    uint32_t arow[NA], bcol[NB];
#pragma unroll
    for (int u = 0; u < NA; ++u) {
        const int m = m0 + RG * (wave * NA + u) + a_r;
        arow[u] = m < M ? (uint32_t)m * (uint32_t)ft.lda * (uint32_t)sizeof(T) + 4u * a_h : kOutOfRange;
    }
#pragma unroll
    for (int v = 0; v < NB; ++v) {
        const int f = 64 * (wave * NB + v) + lane;                // dword of the B stage (unpadded)
        const int n = n0 + (f / EW) % BN;
        bcol[v] = n < N ? (uint32_t)n * (uint32_t)sizeof(T) + 4u * (f % EW) : kOutOfRange;
    }
    const uint32_t ldbb = (uint32_t)ft.ldb * (uint32_t)sizeof(T);

    V4 acc[WBM][WBN];
#pragma unroll
    for (int i = 0; i < WBM; ++i)
#pragma unroll
        for (int j = 0; j < WBN; ++j) acc[i][j] = V4{0, 0, 0, 0};

    // step `st` of the K loop into stage buffer st % NS
    auto issue = [&](int st) {
        const uint32_t sa = lds0 + (uint32_t)((st % NS) * ST_DW) * 4u, sb = sa + A_DW * 4u;
        const int k0 = st * BK;
        const int ka = k0 + a_k;
        const bool kav = ka < K;
#pragma unroll
        for (int u = 0; u < NA; ++u)
            dma_dword(rA, sa + (uint32_t)((wave * NA + u) * AGS) * 4u,
                      kav ? arow[u] + (uint32_t)ka * (uint32_t)sizeof(T) : kOutOfRange);
#pragma unroll
        for (int v = 0; v < NB; ++v) {
            const int x = wave * NB + v;                  // chunk of the B stage
            const int kb = k0 + (64 * x + lane) / EW / BN;
            dma_dword(rB, sb + (uint32_t)(x * BCS) * 4u, kb < K ? bcol[v] + (uint32_t)kb * ldbb : kOutOfRange);
        }
    };

    // per-lane LDS read offsets (dwords within a stage)
    const int c = lane & 15, g = lane >> 4;
    int aoff[WBM], boff[WBN][4];
#pragma unroll
    for (int i = 0; i < WBM; ++i) {
        const int r = wm + i * 16 + c;
        aoff[i] = (r / RG) * AGS + (r % RG) * 16 * EW + 4 * g * EW;
    }
#pragma unroll
    for (int j = 0; j < WBN; ++j)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            // k = 4 g + q: row-major dword of the 16 x BN tile, plus the padding of its chunk
            const int f = ((4 * g + q) * BN + wn + j * 16 + c) * EW;
            boff[j][q] = A_DW + f + (f >> 6) * PB;
        }

#pragma unroll
    for (int p = 0; p < NS - 1; ++p)
        if (p < nsteps) issue(p);
    for (int s = 0; s < nsteps; ++s) {
        // this wave's loads of step s are done once at most `newer` later steps remain in flight
        const int newer = min(nsteps - s - 1, NS - 2);
        if (NS >= 4 && newer >= 2) wait_vm<2 * NL>();
        else if (NS >= 3 && newer >= 1) wait_vm<NL>();
        else wait_vm<0>();
        __syncthreads();
        if (s + NS - 1 < nsteps) issue(s + NS - 1);
        const float *st = sm + (s % NS) * ST_DW;
        T a[WBM][4], b[WBN][4];
#pragma unroll
        for (int i = 0; i < WBM; ++i) {
            // the lane's four consecutive k of its row: EW 16-byte reads
            const f4 lo = *reinterpret_cast<const f4 *>(st + aoff[i]);
            if constexpr (EW == 1) {
                a[i][0] = lo.x; a[i][1] = lo.y; a[i][2] = lo.z; a[i][3] = lo.w;
            } else {
                const f4 hi = *reinterpret_cast<const f4 *>(st + aoff[i] + 4);
                a[i][0] = __builtin_bit_cast(double, f2v{lo.x, lo.y});
                a[i][1] = __builtin_bit_cast(double, f2v{lo.z, lo.w});
                a[i][2] = __builtin_bit_cast(double, f2v{hi.x, hi.y});
                a[i][3] = __builtin_bit_cast(double, f2v{hi.z, hi.w});
            }
        }
#pragma unroll
        for (int j = 0; j < WBN; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) b[j][q] = *reinterpret_cast<const T *>(st + boff[j][q]);
        if constexpr (SPLIT) {
            // a lane's four words are k = 4 g .. 4 g + 3 of its row (column):
            // exactly the four bf16 of one v_mfma_f32_16x16x16_bf16 operand
            s4v ah[WBM], al[WBM], bh[WBN], bl[WBN];
#pragma unroll
            for (int i = 0; i < WBM; ++i) {
                ah[i] = split_hi(a[i][0], a[i][1], a[i][2], a[i][3]);
                al[i] = split_lo(a[i][0], a[i][1], a[i][2], a[i][3]);
            }
#pragma unroll
            for (int j = 0; j < WBN; ++j) {
                bh[j] = split_hi(b[j][0], b[j][1], b[j][2], b[j][3]);
                bl[j] = split_lo(b[j][0], b[j][1], b[j][2], b[j][3]);
            }
#pragma unroll
            for (int i = 0; i < WBM; ++i)
#pragma unroll
                for (int j = 0; j < WBN; ++j) {
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
                }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int i = 0; i < WBM; ++i)
#pragma unroll
                    for (int j = 0; j < WBN; ++j) acc[i][j] = mfma16(a[i][q], b[j][q], acc[i][j]);
        }
    }

    // result rows held by (lane, register r): v_mfma_f64_16x16x4 returns row
    // 4 r + lane/16, v_mfma_f32_16x16x4 and v_mfma_f32_16x16x16_bf16 row
    // 4 (lane/16) + r; column lane % 16
    TC *C = static_cast<TC *>(const_cast<void *>(slots.p[ft.c_slot])) + ft.c_off;
#pragma unroll
    for (int i = 0; i < WBM; ++i)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = EW == 2 ? r * 4 + (lane >> 4) : (lane >> 4) * 4 + r;
            const int gm = m0 + wm + i * 16 + row;
            if (gm >= M) continue;
            TC *Cr = C + (ft.rmap >= 0 ? rowoff[ft.rmap + gm] : (int64_t)gm * ft.ldc);
#pragma unroll
            for (int j = 0; j < WBN; ++j) {
                const int gn = n0 + wn + j * 16 + c;
                if (gn < N) Cr[gn] = (TC)acc[i][j][r];
            }
        }
}

struct GemmArgs {
    Slots sl;
    const GemmItem *it;
    const GemmSeg *sg;
    const GemmTile *tl;
    const int64_t *ro;
    int n;
};

template <typename T, typename TC, int BM, int BN, int WGM, int KDIV>
static void dispatch_shape(bool ta, bool tb, dim3 g, hipStream_t s, const GemmArgs &a) {
    if (!ta && !tb)
        hipLaunchKernelGGL((gemm_kmajor<T, TC, false, false, BM, BN, WGM, KDIV>), g, dim3(NT), 0, s, a.sl, a.it, a.sg, a.tl, a.ro, a.n);
    else if (ta && !tb)
        hipLaunchKernelGGL((gemm_kmajor<T, TC, true, false, BM, BN, WGM, KDIV>), g, dim3(NT), 0, s, a.sl, a.it, a.sg, a.tl, a.ro, a.n);
    else if (!ta && tb)
        hipLaunchKernelGGL((gemm_kmajor<T, TC, false, true, BM, BN, WGM, KDIV>), g, dim3(NT), 0, s, a.sl, a.it, a.sg, a.tl, a.ro, a.n);
    else
        hipLaunchKernelGGL((gemm_kmajor<T, TC, true, true, BM, BN, WGM, KDIV>), g, dim3(NT), 0, s, a.sl, a.it, a.sg, a.tl, a.ro, a.n);
}

// Pipeline depth of the LDS-DMA kernel: two stages (loads one K step ahead)
// keep 8 FP32 workgroups of 64 x 64 resident per CU, which measured faster on
// the H_eff GEMMs than three or four stages at lower occupancy.
constexpr int kDmaStages = 2;
template <typename T, typename TC, int BM, int BN, int WGM, bool SPLIT>
static void dispatch_dma(dim3 g, hipStream_t s, const Slots &sl, const FlatTile *t, const int64_t *ro, int n) {
    hipLaunchKernelGGL((gemm_dma<T, TC, BM, BN, WGM, kDmaStages, SPLIT>), g, dim3(NT), 0, s, sl, t, ro, n);
}
template <typename T, typename TC, bool SPLIT = false>
static void dispatch_dma_shape(TileShape shape, dim3 g, hipStream_t s, const Slots &sl, const FlatTile *t,
                               const int64_t *ro, int n) {
    switch (shape) {
        case TileShape::T128x32_D: dispatch_dma<T, TC, 128, 32, 4, SPLIT>(g, s, sl, t, ro, n); break;
        case TileShape::T64x64_D: dispatch_dma<T, TC, 64, 64, 2, SPLIT>(g, s, sl, t, ro, n); break;
        case TileShape::T32x128_D: dispatch_dma<T, TC, 32, 128, 1, SPLIT>(g, s, sl, t, ro, n); break;
        default: break;
    }
}

template <typename T, typename TC>
static void dispatch_kmajor(TileShape shape, bool ta, bool tb, dim3 g, hipStream_t s, const GemmArgs &a) {
    switch (shape) {
        case TileShape::T64x64: dispatch_shape<T, TC, 64, 64, 2, 1>(ta, tb, g, s, a); break;
        case TileShape::T128x32: dispatch_shape<T, TC, 128, 32, 4, 1>(ta, tb, g, s, a); break;
        case TileShape::T32x128: dispatch_shape<T, TC, 32, 128, 1, 1>(ta, tb, g, s, a); break;
        case TileShape::T128x128: dispatch_shape<T, TC, 128, 128, 2, 1>(ta, tb, g, s, a); break;
        case TileShape::T64x64_K16: dispatch_shape<T, TC, 64, 64, 2, 2>(ta, tb, g, s, a); break;
        case TileShape::T128x32_K16: dispatch_shape<T, TC, 128, 32, 4, 2>(ta, tb, g, s, a); break;
        // FP64 quarter-depth steps (BK = 4) would leave threads without an
        // element of a 32-wide tile; they run at half depth instead
        case TileShape::T64x64_K8: dispatch_shape<T, TC, 64, 64, 2, sizeof(T) == 8 ? 2 : 4>(ta, tb, g, s, a); break;
        case TileShape::T128x32_K8: dispatch_shape<T, TC, 128, 32, 4, sizeof(T) == 8 ? 2 : 4>(ta, tb, g, s, a); break;
        // LDS-DMA pipeline: FP32 non-transposed operands; otherwise the
        // half-depth kernel of the same tile
        // LDS-DMA shapes run through launch_gemm_flat; lists it cannot take
        // (FP64, transposed operands, several segments per item) run the
        // register-staged kernel of the same tile
        case TileShape::T128x32_D: dispatch_shape<T, TC, 128, 32, 4, 2>(ta, tb, g, s, a); break;
        case TileShape::T64x64_D: dispatch_shape<T, TC, 64, 64, 2, 2>(ta, tb, g, s, a); break;
        case TileShape::T32x128_D: dispatch_shape<T, TC, 32, 128, 1, 1>(ta, tb, g, s, a); break;
    }
}

void launch_gemm_flat(GemmPrec prec, TileShape shape, bool c_is_f64, const Slots &slots, const FlatTile *tiles,
                      const int64_t *rowoff, int ntiles, hipStream_t s) {
    if (ntiles <= 0) return;
    const dim3 g(ntiles);
    if (prec == GemmPrec::F64) dispatch_dma_shape<double, double>(shape, g, s, slots, tiles, rowoff, ntiles);
    else if (prec == GemmPrec::BF16X3 && c_is_f64)
        dispatch_dma_shape<float, double, true>(shape, g, s, slots, tiles, rowoff, ntiles);
    else if (prec == GemmPrec::BF16X3) dispatch_dma_shape<float, float, true>(shape, g, s, slots, tiles, rowoff, ntiles);
    else if (c_is_f64) dispatch_dma_shape<float, double>(shape, g, s, slots, tiles, rowoff, ntiles);
    else dispatch_dma_shape<float, float>(shape, g, s, slots, tiles, rowoff, ntiles);
}

void launch_gemm(GemmPrec prec, TileShape shape, bool ta, bool tb, bool c_is_f64, const Slots &slots,
                 const GemmItem *items, const GemmSeg *segs, const GemmTile *tiles, const int64_t *rowoff,
                 int ntiles, hipStream_t s) {
    if (ntiles <= 0) return;
    dim3 grid(ntiles);
    const GemmArgs a{slots, items, segs, tiles, rowoff, ntiles};
    switch (prec) {
        case GemmPrec::F64:
            dispatch_kmajor<double, double>(shape, ta, tb, grid, s, a);
            break;
        case GemmPrec::F32:
            if (c_is_f64) dispatch_kmajor<float, double>(shape, ta, tb, grid, s, a);
            else dispatch_kmajor<float, float>(shape, ta, tb, grid, s, a);
            break;
        case GemmPrec::BF16X3:   // split operands: LDS-DMA lists only (launch_gemm_flat)
            break;
    }
}

}  // namespace pdmrg
