// Bandwidth-bound kernels of the pdmrg library: the MPO (W) stage as a scaled
// sum of strided blocks, diag(H_eff), precision conversions, the FP64 vector
// kernels of the Davidson solver and its small projected eigenproblem.
// Reductions are two-pass with a fixed summation order (no floating-point
// atomics), so results are bitwise reproducible.
#include "kernels.hpp"

#include <algorithm>
#include <stdexcept>
#include <type_traits>

namespace pdmrg {

// A value split for BF16x3: its FP32 rounding f = hi + lo with hi and lo
// bf16 (both rounded to nearest even), packed as one word, hi in the low half.
typedef float pf2 __attribute__((ext_vector_type(2)));
typedef __bf16 pb2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_split(float f) {
    const pf2 x{f, 0.0f};
    const pb2 h = __builtin_convertvector(x, pb2);
    const pb2 l = __builtin_convertvector(x - __builtin_convertvector(h, pf2), pb2);
    return (__builtin_bit_cast(uint32_t, h) & 0xffffu) | (__builtin_bit_cast(uint32_t, l) << 16);
}

// ------------------------------------------------------------ W stage
// One workgroup per tile = a run of kLcChunk consecutive elements of a task's
// rows x cols block in row-major order, so narrow sector blocks keep every
// thread busy.  Each thread owns kLcChunk / 256 elements; the loads of four
// sources are issued together before they are summed (in list order), so a
// task's latency is a quarter of one load chain per source.  Offsets inside a
// block are 32-bit (the list's validation bounds them).
template <typename T, typename TD, int CHUNK>
__global__ __launch_bounds__(256) void lincomb_kernel(Slots slots, const LcTask *__restrict__ tasks,
                                                      const LcSrc *__restrict__ srcs,
                                                      const LcTile *__restrict__ tiles) {
    constexpr int U = CHUNK / 256, J = 4;
    const LcTile tl = tiles[blockIdx.x];
    const LcTask tk = tasks[tl.task];
    // rows * cols < 2^31 (checked when the list is built)
    const unsigned n = (unsigned)tk.rows * (unsigned)tk.cols;
    const unsigned e0 = (unsigned)tl.r0 * CHUNK;
    unsigned rr[U], cc[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const unsigned e = e0 + threadIdx.x + 256 * u;
        ok[u] = e < n;
        const unsigned r = ok[u] ? e / (unsigned)tk.cols : 0u;
        cc[u] = ok[u] ? e - r * (unsigned)tk.cols : 0u;
        rr[u] = r;
    }
    T acc[U];
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u] = 0;
    int j = 0;
    for (; j + J <= tk.nsrc; j += J) {
        T v[J][U], cf[J];
#pragma unroll
        for (int q = 0; q < J; ++q) {
            const LcSrc sj = srcs[tk.src0 + j + q];
            const T *src = static_cast<const T *>(slots.p[sj.slot]) + sj.off;
            cf[q] = (T)sj.coef;
#pragma unroll
            for (int u = 0; u < U; ++u) v[q][u] = ok[u] ? src[rr[u] * (unsigned)sj.ld + cc[u]] : T(0);
        }
#pragma unroll
        for (int q = 0; q < J; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) acc[u] += cf[q] * v[q][u];
    }
    for (; j < tk.nsrc; ++j) {
        const LcSrc sj = srcs[tk.src0 + j];
        const T *src = static_cast<const T *>(slots.p[sj.slot]) + sj.off;
        const T cf = (T)sj.coef;
        T v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = ok[u] ? src[rr[u] * (unsigned)sj.ld + cc[u]] : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] += cf * v[u];
    }
    TD *dst = static_cast<TD *>(const_cast<void *>(slots.p[tk.dst_slot])) + tk.dst_off;
#pragma unroll
    for (int u = 0; u < U; ++u)
        if (ok[u]) {
            if constexpr (std::is_same<TD, uint32_t>::value) dst[rr[u] * (unsigned)tk.ld + cc[u]] = pack_split(acc[u]);
            else dst[rr[u] * (unsigned)tk.ld + cc[u]] = (TD)acc[u];
        }
}

void launch_lincomb(bool f64, int chunk, const Slots &slots, const LcTask *tasks, const LcSrc *srcs,
                    const LcTile *tiles, int ntiles, hipStream_t s) {
    if (ntiles <= 0) return;
    check_grid(ntiles, 256, "W stage");
    const dim3 g(ntiles), b(256);
    if (chunk == kLcChunkSmall) {
        if (f64) hipLaunchKernelGGL((lincomb_kernel<double, double, kLcChunkSmall>), g, b, 0, s, slots, tasks, srcs, tiles);
        else hipLaunchKernelGGL((lincomb_kernel<float, float, kLcChunkSmall>), g, b, 0, s, slots, tasks, srcs, tiles);
    } else {
        if (f64) hipLaunchKernelGGL((lincomb_kernel<double, double, kLcChunk>), g, b, 0, s, slots, tasks, srcs, tiles);
        else hipLaunchKernelGGL((lincomb_kernel<float, float, kLcChunk>), g, b, 0, s, slots, tasks, srcs, tiles);
    }
}

void launch_lincomb_split(int chunk, const Slots &slots, const LcTask *tasks, const LcSrc *srcs,
                          const LcTile *tiles, int ntiles, hipStream_t s) {
    if (ntiles <= 0) return;
    check_grid(ntiles, 256, "W stage");
    const dim3 g(ntiles), b(256);
    if (chunk == kLcChunkSmall)
        hipLaunchKernelGGL((lincomb_kernel<float, uint32_t, kLcChunkSmall>), g, b, 0, s, slots, tasks, srcs, tiles);
    else
        hipLaunchKernelGGL((lincomb_kernel<float, uint32_t, kLcChunk>), g, b, 0, s, slots, tasks, srcs, tiles);
}

void launch_lincomb_f32_f64(int chunk, const Slots &slots, const LcTask *tasks, const LcSrc *srcs,
                            const LcTile *tiles, int ntiles, hipStream_t s) {
    if (ntiles <= 0) return;
    check_grid(ntiles, 256, "W stage");
    const dim3 g(ntiles), b(256);
    if (chunk == kLcChunkSmall)
        hipLaunchKernelGGL((lincomb_kernel<float, double, kLcChunkSmall>), g, b, 0, s, slots, tasks, srcs, tiles);
    else
        hipLaunchKernelGGL((lincomb_kernel<float, double, kLcChunk>), g, b, 0, s, slots, tasks, srcs, tiles);
}

// ------------------------------------------------------------ block dot products
// Workgroup b takes tiles b, b + gridDim.x, ... (grid stride: tile lists can
// outgrow one launch's grid); partial[t] is tile t's sum.
__global__ __launch_bounds__(256) void dot_partial_kernel(Slots slots, int a_slot, int b_slot,
                                                          const DotTask *__restrict__ tasks,
                                                          const DotTile *__restrict__ tiles, int ntiles,
                                                          double *__restrict__ partial) {
    constexpr int U = kDotChunk / 256;
    __shared__ double red[256];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const DotTile tl = tiles[t];
        const DotTask tk = tasks[tl.task];
        const double *a = static_cast<const double *>(slots.p[a_slot]) + tk.a_off;
        const double *b = static_cast<const double *>(slots.p[b_slot]) + tk.b_off;
        const int e0 = tl.chunk * kDotChunk + (int)threadIdx.x;
        double va[U], vb[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int e = e0 + 256 * u;
            va[u] = e < tk.n ? a[e] : 0.0;
            vb[u] = e < tk.n ? b[e] : 0.0;
        }
        double acc = 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u) acc += va[u] * vb[u];
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[t] = red[0];
        __syncthreads();   // red is rewritten by the next tile
    }
}

__global__ void dot_reduce_kernel(const double *__restrict__ partial, const int32_t *__restrict__ t0,
                                  const int32_t *__restrict__ g_of, int ngroups, double *__restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ngroups) return;
    double acc = 0.0;
    for (int t = t0[k]; t < t0[k + 1]; ++t) acc += partial[t];
    out[g_of[k]] = acc;
}

void launch_dot_partials(const Slots &slots, int a_slot, int b_slot, const DotTask *tasks, const DotTile *tiles,
                         int ntiles, double *partial, hipStream_t s) {
    if (ntiles <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(ntiles, kMaxGrid);
    hipLaunchKernelGGL(dot_partial_kernel, dim3(g), dim3(256), 0, s, slots, a_slot, b_slot, tasks, tiles, ntiles,
                       partial);
}

void launch_dot_reduce(const double *partial, const int32_t *t0, const int32_t *g_of, int ngroups, double *out,
                       hipStream_t s) {
    if (ngroups <= 0) return;
    hipLaunchKernelGGL(dot_reduce_kernel, dim3((ngroups + 255) / 256), dim3(256), 0, s, partial, t0, g_of, ngroups,
                       out);
}

// ------------------------------------------------------------ diag(H_eff)
__global__ __launch_bounds__(256) void diag_kernel(Slots slots, const DiagTerm *__restrict__ terms,
                                                   const int32_t *__restrict__ groups) {
    const int g = blockIdx.x;
    const int t0 = groups[g], t1 = groups[g + 1];
    if (t0 == t1) return;
    const DiagTerm head = terms[t0];
    double *out = static_cast<double *>(const_cast<void *>(slots.p[0])) + head.out_off;
    const int r = blockIdx.y;
    if (r >= head.rows) return;
    for (int c = threadIdx.x; c < head.cols; c += 256) {
        double acc = 0.0;
        for (int t = t0; t < t1; ++t) {
            const DiagTerm tm = terms[t];
            const double *L = static_cast<const double *>(slots.p[1]) + tm.l_off;
            const double *R = static_cast<const double *>(slots.p[2]) + tm.r_off;
            acc += tm.coef * L[(int64_t)r * tm.lstride] * R[(int64_t)c * tm.rstride];
        }
        out[(int64_t)r * head.ld + c] = acc;
    }
}

void launch_diag_terms(const Slots &slots, const DiagTerm *terms, const int32_t *groups, int ngroups,
                       int max_rows, hipStream_t s) {
    if (ngroups <= 0 || max_rows <= 0) return;
    hipLaunchKernelGGL(diag_kernel, dim3(ngroups, max_rows), dim3(256), 0, s, slots, terms, groups);
}

// ------------------------------------------------------------ elementwise
__global__ void cvt_d2f(const double *x, float *y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}
__global__ void cvt_d2split(const double *x, uint32_t *y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = pack_split((float)x[i]);
}
__global__ void cvt_f2d(const float *x, double *y, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}
__global__ void fill_kernel(double *x, double v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = v;
}

static dim3 grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 8192) b = 8192;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

void launch_convert_f64_f32(const double *x, float *y, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cvt_d2f, grid_for(n), dim3(256), 0, s, x, y, n);
}
void launch_convert_f64_split(const double *x, uint32_t *y, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cvt_d2split, grid_for(n), dim3(256), 0, s, x, y, n);
}
void launch_convert_f32_f64(const float *x, double *y, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(cvt_f2d, grid_for(n), dim3(256), 0, s, x, y, n);
}
void launch_fill(double *x, double v, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(fill_kernel, grid_for(n), dim3(256), 0, s, x, v, n);
}

__global__ void row_scale_kernel(const double *x, double *y, const int64_t *base, const int32_t *rows,
                                 const int32_t *cols, const int64_t *vbase, const double *scale) {
    const int k = blockIdx.y;
    const int64_t n = (int64_t)rows[k] * cols[k];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / cols[k]);
        y[base[k] + e] = x[base[k] + e] * scale[vbase[k] + r];
    }
}

void launch_row_scale(const double *x, double *y, const int64_t *base, const int32_t *rows,
                      const int32_t *cols, const int64_t *vbase, int nblk, int max_elems,
                      const double *scale, hipStream_t s) {
    if (nblk <= 0 || max_elems <= 0) return;
    dim3 g(std::min(1024, (max_elems + 255) / 256), nblk);
    hipLaunchKernelGGL(row_scale_kernel, g, dim3(256), 0, s, x, y, base, rows, cols, vbase, scale);
}

// ------------------------------------------------------------ Davidson vectors
__device__ __forceinline__ double block_sum(double v, double *sh) {
    // fixed-order tree reduction over 256 threads
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void multidot_kernel(const double *V, int64_t ldv, int nvec, const double *w,
                                                       int64_t n, double *partial) {
    __shared__ double sh[256];
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
    for (int v = 0; v < nvec; ++v) {
        double acc = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) acc += V[v * ldv + i] * w[i];
        acc = block_sum(acc, sh);
        if (threadIdx.x == 0) partial[blockIdx.x * nvec + v] = acc;
    }
}

void launch_multidot(const double *V, int64_t ldv, int nvec, const double *w, int64_t n, double *partial,
                     int nblk, hipStream_t s) {
    if (nvec <= 0) return;
    hipLaunchKernelGGL(multidot_kernel, dim3(nblk), dim3(256), 0, s, V, ldv, nvec, w, n, partial);
}

// one workgroup per vector: strided partial sums, then a fixed-order tree
__global__ __launch_bounds__(256) void reduce_partials_kernel(const double *partial, int nblk, int nvec,
                                                              double *out, int stride) {
    __shared__ double sh[256];
    const int v = blockIdx.x;
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[b * nvec + v];
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) out[(int64_t)v * stride] = acc;
}

void launch_reduce_partials(const double *partial, int nblk, int nvec, double *out, int stride,
                            hipStream_t s) {
    if (nvec <= 0) return;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(nvec), dim3(256), 0, s, partial, nblk, nvec, out, stride);
}

__global__ void combine_kernel(const double *V, int64_t ldv, int nvec, const double *c, double *y, int64_t n,
                               double beta, double sign) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int v = 0; v < nvec; ++v) acc += c[v] * V[v * ldv + i];
        // beta = 0: y is output only (its old contents, possibly NaN, are not read)
        y[i] = beta == 0.0 ? sign * acc : beta * y[i] + sign * acc;
    }
}

void launch_combine(const double *V, int64_t ldv, int nvec, const double *c, double *y, int64_t n, double beta,
                    hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, grid_for(n), dim3(256), 0, s, V, ldv, nvec, c, y, n, beta, 1.0);
}
void launch_subtract_combine(const double *V, int64_t ldv, int nvec, const double *c, double *y, int64_t n,
                             hipStream_t s) {
    hipLaunchKernelGGL(combine_kernel, grid_for(n), dim3(256), 0, s, V, ldv, nvec, c, y, n, 1.0, -1.0);
}

__global__ void residual_kernel(const double *hx, const double *x, const double *theta, double *r, int64_t n) {
    const double th = *theta;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = hx[i] - th * x[i];
}
void launch_residual(const double *hx, const double *x, const double *theta, double *r, int64_t n,
                     hipStream_t s) {
    hipLaunchKernelGGL(residual_kernel, grid_for(n), dim3(256), 0, s, hx, x, theta, r, n);
}

__global__ void precond_kernel(const double *r, const double *diag, const double *theta, double *t, int64_t n) {
    const double th = *theta;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double den = diag[i] - th;
        if (fabs(den) < 1e-8) den = copysign(1e-8, den);
        t[i] = r[i] / den;
    }
}
void launch_precond(const double *r, const double *diag, const double *theta, double *t, int64_t n,
                    hipStream_t s) {
    hipLaunchKernelGGL(precond_kernel, grid_for(n), dim3(256), 0, s, r, diag, theta, t, n);
}

__global__ void scale_inv_sqrt_kernel(const double *x, const double *nrm2, double *y, int64_t n) {
    const double f = 1.0 / sqrt(*nrm2);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * f;
}
void launch_scale_by_inv_sqrt(const double *x, const double *nrm2, double *y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(scale_inv_sqrt_kernel, grid_for(n), dim3(256), 0, s, x, nrm2, y, n);
}

// ------------------------------------------------------------ fused Davidson passes
// Block b owns the contiguous element range [b chunk, (b + 1) chunk); every
// thread keeps one running sum per output, then the sums of a block are
// reduced in a fixed order (lanes by xor-shuffle, the 4 waves in LDS).
template <int NO>
__device__ __forceinline__ void block_store_sums(double (&acc)[NO], int nout, double *row) {
    __shared__ double sh[4][NO];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NO; ++v) {
        if (v < nout) {   // uniform over the block
            double x = acc[v];
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
            if (lane == 0) sh[wave][v] = x;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nout) {
        const int v = threadIdx.x;
        row[v] = ((sh[0][v] + sh[1][v]) + sh[2][v]) + sh[3][v];
    }
}

__device__ __forceinline__ void block_range(int64_t n, int64_t &i0, int64_t &i1) {
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    i0 = blockIdx.x * chunk;
    i1 = min(n, i0 + chunk);
}

template <int KM>
__global__ __launch_bounds__(256) void dav_ritz_kernel(const double *__restrict__ V, const double *__restrict__ HV,
                                                       int64_t ldv, int k, const double *__restrict__ c,
                                                       const double *__restrict__ theta,
                                                       const double *__restrict__ diag, double *__restrict__ X,
                                                       double *__restrict__ HX, double *__restrict__ R,
                                                       double *__restrict__ T, int64_t n, double *partial) {
    const double th = *theta;
    double cc[KM], acc[KM + 1];
#pragma unroll
    for (int v = 0; v < KM; ++v) cc[v] = v < k ? c[v] : 0.0;
#pragma unroll
    for (int v = 0; v <= KM; ++v) acc[v] = 0.0;
    int64_t i0, i1;
    block_range(n, i0, i1);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        double vv[KM], x = 0.0, hx = 0.0;
#pragma unroll
        for (int v = 0; v < KM; ++v)
            if (v < k) {
                vv[v] = V[v * ldv + i];
                x += cc[v] * vv[v];
            }
#pragma unroll
        for (int v = 0; v < KM; ++v)
            if (v < k) hx += cc[v] * HV[v * ldv + i];
        const double r = hx - th * x;
        double den = diag[i] - th;
        if (fabs(den) < 1e-8) den = copysign(1e-8, den);
        const double t = r / den;
        X[i] = x;
        HX[i] = hx;
        R[i] = r;
        T[i] = t;
        acc[0] += r * r;
#pragma unroll
        for (int v = 0; v < KM; ++v)
            if (v < k) acc[v + 1] += vv[v] * t;
    }
    block_store_sums<KM + 1>(acc, k + 1, partial + (int64_t)blockIdx.x * (k + 1));
}

template <int KM>
__global__ __launch_bounds__(256) void dav_sub_dot_kernel(const double *__restrict__ V, int64_t ldv, int k,
                                                          const double *__restrict__ d, double *__restrict__ T,
                                                          int64_t n, int with_dots, double *partial) {
    double dd[KM], acc[KM];
#pragma unroll
    for (int v = 0; v < KM; ++v) {
        dd[v] = v < k ? d[v] : 0.0;
        acc[v] = 0.0;
    }
    int64_t i0, i1;
    block_range(n, i0, i1);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        double vv[KM], a = 0.0;
#pragma unroll
        for (int v = 0; v < KM; ++v)
            if (v < k) {
                vv[v] = V[v * ldv + i];
                a += dd[v] * vv[v];
            }
        const double t = T[i] - a;
        T[i] = t;
        if (with_dots) {
#pragma unroll
            for (int v = 0; v < KM; ++v)
                if (v < k) acc[v] += vv[v] * t;
        } else {
            acc[0] += t * t;
        }
    }
    const int nout = with_dots ? k : 1;
    block_store_sums<KM>(acc, nout, partial + (int64_t)blockIdx.x * nout);
}

template <int KM>
__global__ __launch_bounds__(256) void dav_ext_gram_kernel(const double *__restrict__ V,
                                                           const double *__restrict__ HV, int64_t ldv, int k,
                                                           int64_t n, double *partial) {
    double acc[2 * KM + 1];
#pragma unroll
    for (int v = 0; v <= 2 * KM; ++v) acc[v] = 0.0;
    int64_t i0, i1;
    block_range(n, i0, i1);
    for (int64_t i = i0 + threadIdx.x; i < i1; i += 256) {
        const double vk = V[k * ldv + i], hk = HV[k * ldv + i];
#pragma unroll
        for (int v = 0; v < KM; ++v)
            if (v < k) {
                acc[v] += V[v * ldv + i] * hk;
                acc[KM + 1 + v] += HV[v * ldv + i] * vk;
            }
        acc[KM] += vk * hk;
    }
    // row of 2 KM + 1 sums: [V_v.HV_k (v < k) ..., V_k.HV_k at KM, HV_v.V_k at KM + 1 + v]
    block_store_sums<2 * KM + 1>(acc, 2 * KM + 1, partial + (int64_t)blockIdx.x * (2 * KM + 1));
}

__global__ void dav_g_scatter_kernel(double *G, int ld, int k, int km, const double *dots, int exact_row) {
    const int v = threadIdx.x;
    if (v < k) G[(int64_t)v * ld + k] = dots[v];
    if (v == k) G[(int64_t)k * ld + k] = dots[km];
    if (v < k) G[(int64_t)k * ld + v] = dots[km + 1 + v];
    __syncthreads();
    if (exact_row && k > 0 && v == 0) G[k] = G[(int64_t)k * ld];
}

void launch_dav_ritz(const double *V, const double *HV, int64_t ldv, int k, const double *c, const double *theta,
                     const double *diag, double *x, double *hx, double *r, double *t, int64_t n, double *partial,
                     int nblk, hipStream_t s) {
    if (k < 1 || k > kDavFused) throw std::invalid_argument("dav_ritz: k out of range");
    if (k <= 8)
        hipLaunchKernelGGL(dav_ritz_kernel<8>, dim3(nblk), dim3(256), 0, s, V, HV, ldv, k, c, theta, diag, x, hx,
                           r, t, n, partial);
    else
        hipLaunchKernelGGL(dav_ritz_kernel<kDavFused>, dim3(nblk), dim3(256), 0, s, V, HV, ldv, k, c, theta, diag,
                           x, hx, r, t, n, partial);
}
void launch_dav_sub_dot(const double *V, int64_t ldv, int k, const double *d, double *t, int64_t n,
                        bool with_dots, double *partial, int nblk, hipStream_t s) {
    if (k < 1 || k > kDavFused) throw std::invalid_argument("dav_sub_dot: k out of range");
    if (k <= 8)
        hipLaunchKernelGGL(dav_sub_dot_kernel<8>, dim3(nblk), dim3(256), 0, s, V, ldv, k, d, t, n, (int)with_dots,
                           partial);
    else
        hipLaunchKernelGGL(dav_sub_dot_kernel<kDavFused>, dim3(nblk), dim3(256), 0, s, V, ldv, k, d, t, n,
                           (int)with_dots, partial);
}
int dav_ext_gram_width(int k) { return k < 8 ? 8 : kDavFused; }
void launch_dav_ext_gram(const double *V, const double *HV, int64_t ldv, int k, int64_t n, double *partial,
                         int nblk, hipStream_t s) {
    if (k < 0 || k >= kDavFused) throw std::invalid_argument("dav_ext_gram: k out of range");
    if (k < 8)
        hipLaunchKernelGGL(dav_ext_gram_kernel<8>, dim3(nblk), dim3(256), 0, s, V, HV, ldv, k, n, partial);
    else
        hipLaunchKernelGGL(dav_ext_gram_kernel<kDavFused>, dim3(nblk), dim3(256), 0, s, V, HV, ldv, k, n, partial);
}
void launch_dav_g_scatter(double *G, int ld, int k, const double *dots, bool exact_row, hipStream_t s) {
    hipLaunchKernelGGL(dav_g_scatter_kernel, dim3(1), dim3(64), 0, s, G, ld, k, dav_ext_gram_width(k), dots,
                       (int)exact_row);
}

// ------------------------------------------------------------ projected eigenproblem
// Cyclic Jacobi with the round-robin (circle) ordering: each round rotates
// n/2 disjoint index pairs, first their columns (A J, V J), then their rows
// (J^T A).  One wave64; k <= 64.
constexpr int SE_MAX = 64;

__global__ __launch_bounds__(64) void small_eig_kernel(const double *G, int k, int ld, double *theta_out,
                                                       double *c_out) {
    __shared__ double A[SE_MAX][SE_MAX + 1];
    __shared__ double V[SE_MAX][SE_MAX + 1];
    __shared__ double rc[SE_MAX / 2], rs[SE_MAX / 2];
    __shared__ int rp[SE_MAX / 2], rq[SE_MAX / 2];
    __shared__ double red[64];
    const int l = threadIdx.x;
    for (int i = 0; i < k; ++i)
        for (int j = l; j < k; j += 64) {
            A[i][j] = 0.5 * (G[i * ld + j] + G[j * ld + i]);
            V[i][j] = (i == j) ? 1.0 : 0.0;
        }
    __syncthreads();
    const int n = (k % 2) ? k + 1 : k;   // players, one dummy if k is odd
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0, dia = 0.0;
        for (int i = 0; i < k; ++i)
            for (int j = l; j < k; j += 64) {
                if (i != j) off += A[i][j] * A[i][j];
                else dia += A[i][j] * A[i][j];
            }
        red[l] = off;
        __syncthreads();
        if (l == 0) {
            double so = 0.0;
            for (int i = 0; i < 64; ++i) so += red[i];
            red[0] = so;
        }
        __syncthreads();
        const double soff = red[0];
        __syncthreads();
        red[l] = dia;
        __syncthreads();
        if (l == 0) {
            double sd = 0.0;
            for (int i = 0; i < 64; ++i) sd += red[i];
            red[0] = sd;
        }
        __syncthreads();
        const double sdia = red[0];
        __syncthreads();
        if (soff <= 1e-30 * sdia || soff == 0.0) break;
        for (int r = 0; r < n - 1; ++r) {
            if (l < n / 2) {
                int p = (l == 0) ? n - 1 : (r + l) % (n - 1);
                int q = (r - l + (n - 1)) % (n - 1);
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < k && p < k && A[p][q] != 0.0) {
                    const double tau = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                    const double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                    c = 1.0 / sqrt(1.0 + t * t);
                    s = t * c;
                }
                rp[l] = p; rq[l] = q; rc[l] = c; rs[l] = s;
            }
            __syncthreads();
            // columns: A J and V J
            for (int e = l; e < (n / 2) * k; e += 64) {
                const int pr = e / k, i = e % k;
                const int p = rp[pr], q = rq[pr];
                if (q >= k) continue;
                const double c = rc[pr], s = rs[pr];
                const double ap = A[i][p], aq = A[i][q];
                A[i][p] = c * ap - s * aq;
                A[i][q] = s * ap + c * aq;
                const double vp = V[i][p], vq = V[i][q];
                V[i][p] = c * vp - s * vq;
                V[i][q] = s * vp + c * vq;
            }
            __syncthreads();
            // rows: J^T A
            for (int e = l; e < (n / 2) * k; e += 64) {
                const int pr = e / k, j = e % k;
                const int p = rp[pr], q = rq[pr];
                if (q >= k) continue;
                const double c = rc[pr], s = rs[pr];
                const double ap = A[p][j], aq = A[q][j];
                A[p][j] = c * ap - s * aq;
                A[q][j] = s * ap + c * aq;
            }
            __syncthreads();
        }
    }
    if (l == 0) {
        int best = 0;
        for (int i = 1; i < k; ++i)
            if (A[i][i] < A[best][best]) best = i;
        red[0] = A[best][best];
        red[1] = (V[0][best] < 0.0) ? -1.0 : 1.0;
        rp[0] = best;
    }
    __syncthreads();
    const int best = rp[0];
    const double sg = red[1];
    for (int i = l; i < k; i += 64) c_out[i] = sg * V[i][best];
    if (l == 0) theta_out[0] = red[0];
}

void launch_small_eig(const double *G, int k, int ld, double *theta_out, double *c_out, hipStream_t s) {
    hipLaunchKernelGGL(small_eig_kernel, dim3(1), dim3(64), 0, s, G, k, ld, theta_out, c_out);
}

// ------------------------------------------------------------ local measurements
// Grid stride over the tiles, as dot_partial_kernel.
__global__ __launch_bounds__(256) void seg_dot_kernel(const SegDot *__restrict__ tasks,
                                                      const SegTile *__restrict__ tiles, int ntiles,
                                                      double *__restrict__ partial) {
    __shared__ double red[256];
    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const SegTile tl = tiles[t];
        const SegDot tk = tasks[tl.task];
        const int nr = min(kSegRows, tk.rows - tl.r0);
        const int n = nr * tk.width;
        double acc = 0.0;
        for (int e = threadIdx.x; e < n; e += 256) {
            const int r = tl.r0 + e / tk.width, c = e % tk.width;
            const double *row = tk.x + (int64_t)r * tk.ld;
            acc += row[tk.ca + c] * row[tk.cb + c];
        }
        red[threadIdx.x] = acc;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[t] = red[0];
        __syncthreads();
    }
}

void launch_seg_dot_partials(const SegDot *tasks, const SegTile *tiles, int ntiles, double *partial, hipStream_t s) {
    if (ntiles <= 0) return;
    const unsigned g = (unsigned)std::min<int64_t>(ntiles, kMaxGrid);
    hipLaunchKernelGGL(seg_dot_kernel, dim3(g), dim3(256), 0, s, tasks, tiles, ntiles, partial);
}

__global__ void set_identity_kernel(const SqBlock *__restrict__ blocks) {
    const SqBlock b = blocks[blockIdx.y];
    const int64_t n2 = (int64_t)b.n * b.n;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n2; e += (int64_t)gridDim.x * blockDim.x)
        b.p[e] = (e / b.n == e % b.n) ? 1.0 : 0.0;
}

void launch_set_identity(const SqBlock *blocks, int nblocks, int max_n, hipStream_t s) {
    if (nblocks <= 0 || max_n <= 0) return;
    const int g = (int)std::min<int64_t>(1024, ((int64_t)max_n * max_n + 255) / 256);
    hipLaunchKernelGGL(set_identity_kernel, dim3(g, nblocks), dim3(256), 0, s, blocks);
}

__global__ __launch_bounds__(256) void trace_sum_kernel(const SqBlock *__restrict__ blocks, int nblocks,
                                                        double *__restrict__ out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int k = 0; k < nblocks; ++k) {
        const SqBlock b = blocks[k];
        for (int r = threadIdx.x; r < b.n; r += 256) acc += b.p[(int64_t)r * b.n + r];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

void launch_trace_sum(const SqBlock *blocks, int nblocks, double *out, hipStream_t s) {
    hipLaunchKernelGGL(trace_sum_kernel, dim3(1), dim3(256), 0, s, blocks, nblocks, out);
}

}  // namespace pdmrg
