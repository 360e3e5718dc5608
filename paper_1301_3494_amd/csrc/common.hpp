// Shared host-side definitions of the pdmrg library: errors, bonds, layouts
// of the block-sparse tensors (see include/pdmrg.h) and device buffers.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pdmrg.h"

namespace pdmrg {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define PD_REQUIRE(cond, code, msg)                                              \
    do {                                                                         \
        if (!(cond)) throw ::pdmrg::Error((code), std::string(msg));             \
    } while (0)

#define HIP_OK(expr)                                                             \
    do {                                                                         \
        hipError_t e_ = (expr);                                                  \
        if (e_ != hipSuccess)                                                    \
            throw ::pdmrg::Error(PDMRG_EHIP, std::string(#expr) + ": " +        \
                                                 hipGetErrorString(e_));          \
    } while (0)

void set_last_error(const std::string &msg);

// ---------------------------------------------------------------- bonds
struct Bond {
    std::vector<int> q, dim;
    std::vector<int64_t> off;   // first state of each sector in bond order
    int total = 0;

    Bond() = default;
    Bond(const std::vector<int> &qs, const std::vector<int> &dims);
    static Bond from(const pdmrg_bond *b);
    int find(int charge) const;   // sector index or -1
    int dim_of(int charge) const { int k = find(charge); return k < 0 ? 0 : dim[k]; }
    int nsec() const { return (int)q.size(); }
    bool operator==(const Bond &o) const { return q == o.q && dim == o.dim; }
};

struct Phys {
    std::vector<int> q;
    int d() const { return (int)q.size(); }
    static Phys from(const pdmrg_phys *p);
};

// ---------------------------------------------------------------- layouts
// SITE / TWO_SITE: one row-major block per left sector.
struct SiteLayout {
    int nphys = 0;                   // d (SITE) or d*d (TWO_SITE)
    std::vector<int64_t> base;       // per left sector
    std::vector<int> rows, cols;     // per left sector
    std::vector<int> colo;           // [nsec_left * nphys]: column offset or -1
    std::vector<int> width;          // [nsec_left * nphys]: segment width (0 if absent)
    int64_t size = 0;
};
SiteLayout site_layout(const Bond &bl, const Bond &br, const Phys &p);
SiteLayout two_site_layout(const Bond &bl, const Bond &br, const Phys &p);

// ENV_L / ENV_R: one row-major block per ket (L) or bra (R) sector; rows grouped
// by channel.
struct EnvLayout {
    int D = 0;
    std::vector<int64_t> base;       // per sector
    std::vector<int> rows, cols;     // per sector (cols = dim of the sector)
    std::vector<int> rowo;           // [nsec * D]: row offset of channel w or -1
    int64_t size = 0;
};
EnvLayout env_l_layout(const Bond &b, const std::vector<int> &deltas);
EnvLayout env_r_layout(const Bond &b, const std::vector<int> &deltas);

// ---------------------------------------------------------------- MPO site
struct MpoSite {
    int Dl = 0, Dr = 0, d = 0;
    std::vector<double> W;           // [Dl][d][d][Dr]
    std::vector<int> dl, dr;
    double at(int wl, int s, int t, int wr) const {
        return W[(((size_t)wl * d + s) * d + t) * Dr + wr];
    }
    static MpoSite from(const pdmrg_mpo_site *s);
};

// ---------------------------------------------------------------- device memory
// Bytes the caching allocator reserves for a request of n bytes.
size_t size_class(size_t n);
// Device bytes handed out by the allocator and not yet released (current and
// peak since the last reset), and bytes held in its cache.
void alloc_stats(int64_t *in_use, int64_t *peak, int64_t *cached);
void alloc_reset_peak();
// pdmrg_set_alloc_poison: fill buffers with NaN bytes as they are handed out
extern std::atomic<bool> g_alloc_poison;

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t n) { alloc(n); }
    ~DevBuf() { release(); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : ptr(o.ptr), bytes(o.bytes) { o.ptr = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); ptr = o.ptr; bytes = o.bytes; o.ptr = nullptr; o.bytes = 0; }
        return *this;
    }
    void alloc(size_t n);
    void ensure(size_t n) { if (n > bytes) { release(); alloc(n); } }
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

template <class T>
void upload(DevBuf &buf, const std::vector<T> &v, hipStream_t s) {
    buf.ensure(std::max<size_t>(v.size() * sizeof(T), 16));
    if (!v.empty()) HIP_OK(hipMemcpyAsync(buf.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Host worker threads for independent jobs of one context (the regions of a
// half-sweep, the merges of one merge phase, groups of correlators).  Threads
// are created on first use and live as long as the context, so a sweep does
// not create and tear down threads per phase; each one selects the context's
// device before every job.
class WorkerPool {
public:
    explicit WorkerPool(int device) : device_(device) {}
    ~WorkerPool();
    WorkerPool(const WorkerPool &) = delete;
    WorkerPool &operator=(const WorkerPool &) = delete;
    // fn(k) for k = 0 .. n-1, job k on worker k; returns once every job has
    // returned.  fn must not throw (jobs report errors through their own
    // records).
    void run(int n, const std::function<void(int)> &fn);

private:
    void loop(int k);
    int device_;
    std::mutex mu_;
    std::condition_variable cv_work_, cv_done_;
    std::vector<std::thread> threads_;
    std::vector<const std::function<void(int)> *> job_;
    std::vector<char> ready_;
    int pending_ = 0;
    bool quit_ = false;
};

}  // namespace pdmrg

// Events per timed heff_apply: before stage 1, the W stage, the stage-3 GEMM,
// the split-K reduction, and after it.
constexpr int kTimingEvents = 5;

struct pdmrg_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // H_eff stage timing: 4 events per heff_apply (before stage 1, 2, 3, after),
    // recorded without synchronisation and summed when queried.
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    int64_t n_timed = 0;
    pdmrg::DevBuf ws_dav;           // Davidson basis and scalars
    pdmrg::DevBuf ws_env;           // environment-update intermediates
    pdmrg::DevBuf ws_merge;         // merge: V-scaled right tensor
    pdmrg::DevBuf ws_svd;           // SVD work space
    pdmrg::DevBuf ws_grad;          // gradient intermediates
    // Tile-shape autotuning of H_eff plans: 0 cost model, 1 measured and
    // cached per block signature, 2 = 1 plus a log line per tuned plan.
    int autotune = 0;
    // Per-region contexts of concurrent sweeps (own stream and work space),
    // created on first use and destroyed with this context; their host
    // threads come from `pool`.
    std::vector<pdmrg_ctx *> sub;
    std::unique_ptr<pdmrg::WorkerPool> pool;
    bool owns_stream = false;
    // Environment recompute stride of sweeps and measurement sweeps on this
    // context (pdmrg_ctx_set_env_stride; <= 1: keep every environment).
    int env_stride = 0;
    int verbose = 0;   // progress lines on stderr
    // Householder QR preconditioning of the truncation SVD's Jacobi iteration
    // (pdmrg_ctx_set_svd_precondition): 0 off, 1 blocks of at least 64 rows,
    // 2 every block (up to rows of 2048).
    int svd_precond = 1;
    // heff_apply through captured graphs (replayed on `stream`); the capture
    // happens on cap_stream, created on first use.
    bool graphs = false;
    hipStream_t cap_stream = nullptr;
};
