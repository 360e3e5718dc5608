// Host bookkeeping of U(1) block-sparse tensors: sector tables and the block
// layouts declared in include/pdmrg.h.
#include "common.hpp"

#include <atomic>
#include <mutex>

namespace pdmrg {

static thread_local std::string g_last_error;
void set_last_error(const std::string &msg) { g_last_error = msg; }
const char *last_error_cstr() { return g_last_error.c_str(); }

Bond::Bond(const std::vector<int> &qs, const std::vector<int> &dims) : q(qs), dim(dims) {
    PD_REQUIRE(q.size() == dim.size(), PDMRG_EINVAL, "bond: charge / dimension count mismatch");
    off.resize(q.size());
    int64_t o = 0;
    for (size_t k = 0; k < q.size(); ++k) {
        PD_REQUIRE(dim[k] > 0, PDMRG_EINVAL, "bond: sector dimension must be positive");
        PD_REQUIRE(k == 0 || q[k] > q[k - 1], PDMRG_EINVAL, "bond: charges must be strictly ascending");
        off[k] = o;
        o += dim[k];
    }
    PD_REQUIRE(o < (1 << 30), PDMRG_EINVAL, "bond: dimension too large");
    total = (int)o;
}

Bond Bond::from(const pdmrg_bond *b) {
    PD_REQUIRE(b != nullptr && b->nsec >= 0, PDMRG_EINVAL, "bond: null descriptor");
    PD_REQUIRE(b->nsec == 0 || (b->q && b->dim), PDMRG_EINVAL, "bond: null arrays");
    return Bond(std::vector<int>(b->q, b->q + b->nsec), std::vector<int>(b->dim, b->dim + b->nsec));
}

int Bond::find(int charge) const {
    auto it = std::lower_bound(q.begin(), q.end(), charge);
    if (it == q.end() || *it != charge) return -1;
    return (int)(it - q.begin());
}

Phys Phys::from(const pdmrg_phys *p) {
    PD_REQUIRE(p != nullptr && p->d > 0 && p->q != nullptr, PDMRG_EINVAL, "phys: bad descriptor");
    Phys r;
    r.q.assign(p->q, p->q + p->d);
    return r;
}

MpoSite MpoSite::from(const pdmrg_mpo_site *s) {
    PD_REQUIRE(s && s->W && s->dl && s->dr && s->Dl > 0 && s->Dr > 0 && s->d > 0, PDMRG_EINVAL,
               "mpo site: bad descriptor");
    MpoSite m;
    m.Dl = s->Dl; m.Dr = s->Dr; m.d = s->d;
    m.W.assign(s->W, s->W + (size_t)s->Dl * s->d * s->d * s->Dr);
    m.dl.assign(s->dl, s->dl + s->Dl);
    m.dr.assign(s->dr, s->dr + s->Dr);
    return m;
}

static SiteLayout generic_site_layout(const Bond &bl, const Bond &br, const Phys &p, bool two) {
    const int d = p.d();
    SiteLayout L;
    L.nphys = two ? d * d : d;
    const int ns = bl.nsec();
    L.base.resize(ns);
    L.rows.resize(ns);
    L.cols.resize(ns);
    L.colo.assign((size_t)ns * L.nphys, -1);
    L.width.assign((size_t)ns * L.nphys, 0);
    int64_t o = 0;
    for (int i = 0; i < ns; ++i) {
        int c = 0;
        for (int s = 0; s < L.nphys; ++s) {
            const int dq = two ? p.q[s / d] + p.q[s % d] : p.q[s];
            const int k = br.find(bl.q[i] + dq);
            if (k < 0) continue;
            L.colo[(size_t)i * L.nphys + s] = c;
            L.width[(size_t)i * L.nphys + s] = br.dim[k];
            c += br.dim[k];
        }
        L.base[i] = o;
        L.rows[i] = bl.dim[i];
        L.cols[i] = c;
        o += (int64_t)bl.dim[i] * c;
    }
    L.size = o;
    return L;
}

SiteLayout site_layout(const Bond &bl, const Bond &br, const Phys &p) {
    return generic_site_layout(bl, br, p, false);
}
SiteLayout two_site_layout(const Bond &bl, const Bond &br, const Phys &p) {
    return generic_site_layout(bl, br, p, true);
}

static EnvLayout generic_env_layout(const Bond &b, const std::vector<int> &deltas, int sign) {
    // L (sign +1): per ket sector q', rows = bra states of q' + delta_w;
    // R (sign -1): per bra sector q, rows = ket states of q - delta_w.
    EnvLayout E;
    E.D = (int)deltas.size();
    const int ns = b.nsec();
    E.base.resize(ns);
    E.rows.resize(ns);
    E.cols.resize(ns);
    E.rowo.assign((size_t)ns * E.D, -1);
    int64_t o = 0;
    for (int j = 0; j < ns; ++j) {
        int r = 0;
        for (int w = 0; w < E.D; ++w) {
            const int k = b.find(b.q[j] + sign * deltas[w]);
            if (k < 0) continue;
            E.rowo[(size_t)j * E.D + w] = r;
            r += b.dim[k];
        }
        E.base[j] = o;
        E.rows[j] = r;
        E.cols[j] = b.dim[j];
        o += (int64_t)r * b.dim[j];
    }
    E.size = o;
    return E;
}

EnvLayout env_l_layout(const Bond &b, const std::vector<int> &deltas) { return generic_env_layout(b, deltas, +1); }
EnvLayout env_r_layout(const Bond &b, const std::vector<int> &deltas) { return generic_env_layout(b, deltas, -1); }

// Caching device allocator behind DevBuf.  Sizes are rounded up to a size
// class: powers of two up to 1 MiB, above that multiples of one eighth of the
// power of two below the request (at most 12.5 % over the request, so a
// 1.8 GB environment takes 1.88 GB, not 2 GiB).  Released blocks go to a
// pending list and become reusable only after one device-wide
// synchronisation, so a block can never be handed out while a kernel launched
// before its release still uses it.  That synchronisation waits for every
// stream (concurrent regions included), so it is taken only once the pending
// blocks hold kRecycleBytes; below that a miss allocates a new block.  Cached
// blocks are kept until the process ends.
//
// The mutex guards only the host lists: hipMalloc, hipFree and the device
// synchronisation run with it released, so a thread that allocates never
// holds up the HIP calls of the other region threads.  Blocks moved out of
// the pending list are owned by the thread that synchronises; ones released
// meanwhile stay pending for the next round.
std::atomic<bool> g_alloc_poison{false};

namespace {
std::mutex g_cache_mu;   // the allocator serves every host thread of the process

// debugging aid: NaN bytes in a buffer about to be handed out
void poison(void *ptr, size_t bytes) {
    if (!g_alloc_poison.load(std::memory_order_relaxed)) return;
    HIP_OK(hipDeviceSynchronize());
    HIP_OK(hipMemset(ptr, 0xFF, bytes));
    HIP_OK(hipDeviceSynchronize());
}
constexpr size_t kRecycleBytes = size_t(2) << 30;
using BlockMap = std::map<std::pair<int, size_t>, std::vector<void *>>;
struct DeviceCache {
    BlockMap free_, pending_;
    size_t pending_bytes = 0;
    int64_t in_use = 0, peak = 0, cached = 0;   // bytes (size classes)
};
DeviceCache &cache() {
    static DeviceCache *c = new DeviceCache();   // never destroyed: no hipFree after runtime teardown
    return *c;
}
}  // namespace

size_t size_class(size_t n) {
    size_t c = 256;
    while (c < n && c < (size_t(1) << 20)) c <<= 1;
    if (c >= n) return c;
    size_t p = size_t(1) << 20;
    while (p * 2 <= n) p <<= 1;
    const size_t step = p / 8;
    return (n + step - 1) / step * step;
}

namespace {
// under g_cache_mu: a cached block of class `cls` on `dev`, or null
void *take_free(DeviceCache &c, int dev, size_t cls) {
    auto it = c.free_.find(std::make_pair(dev, cls));
    if (it == c.free_.end() || it->second.empty()) return nullptr;
    void *p = it->second.back();
    it->second.pop_back();
    return p;
}
void merge_into(BlockMap &dst, BlockMap &src) {
    for (auto &kv : src) {
        auto &d = dst[kv.first];
        d.insert(d.end(), kv.second.begin(), kv.second.end());
    }
    src.clear();
}
}  // namespace

void DevBuf::alloc(size_t n) {
    if (n == 0) n = 16;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    const size_t cls = size_class(n);
    DeviceCache &c = cache();
    void *p = nullptr;
    BlockMap recycled;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        p = take_free(c, dev, cls);
        if (!p && c.pending_bytes >= kRecycleBytes) {
            recycled.swap(c.pending_);
            c.pending_bytes = 0;
        }
    }
    if (!recycled.empty()) {
        // every kernel that used these blocks was launched before they were
        // released, hence before this synchronisation
        HIP_OK(hipDeviceSynchronize());
        std::lock_guard<std::mutex> lk(g_cache_mu);
        merge_into(c.free_, recycled);
        p = take_free(c, dev, cls);
    }
    if (!p) {
        hipError_t e = hipMalloc(&p, cls);
        if (e != hipSuccess) {
            // out of memory: give every cached block back to the runtime and retry once
            (void)hipGetLastError();
            BlockMap all;
            {
                std::lock_guard<std::mutex> lk(g_cache_mu);
                merge_into(all, c.free_);
                merge_into(all, c.pending_);
                c.pending_bytes = 0;
            }
            HIP_OK(hipDeviceSynchronize());
            for (auto &kv : all)
                for (void *q : kv.second) (void)hipFree(q);
            p = nullptr;
            e = hipMalloc(&p, cls);
        }
        if (e != hipSuccess) {
            ptr = nullptr;
            bytes = 0;
            throw Error(PDMRG_ENOMEM, "hipMalloc of " + std::to_string(cls) + " bytes failed: " + hipGetErrorString(e));
        }
    }
    ptr = p;
    bytes = cls;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        c.in_use += (int64_t)cls;
        c.peak = std::max(c.peak, c.in_use);
    }
    poison(ptr, cls);
}

void alloc_stats(int64_t *in_use, int64_t *peak, int64_t *cached) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    DeviceCache &c = cache();
    int64_t held = 0;
    for (auto *m : {&c.free_, &c.pending_})
        for (auto &kv : *m) held += (int64_t)kv.first.second * (int64_t)kv.second.size();
    if (in_use) *in_use = c.in_use;
    if (peak) *peak = c.peak;
    if (cached) *cached = held;
}

void alloc_reset_peak() {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    cache().peak = cache().in_use;
}

void DevBuf::release() {
    if (ptr) {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            DeviceCache &c = cache();
            c.pending_[std::make_pair(dev, bytes)].push_back(ptr);
            c.pending_bytes += bytes;
            c.in_use -= (int64_t)bytes;
        }
    }
    ptr = nullptr;
    bytes = 0;
}

void check_grid(int64_t blocks, int threads, const char *what) {
    PD_REQUIRE(blocks >= 0 && blocks * (int64_t)threads < (int64_t(1) << 32), PDMRG_ESHAPE,
               std::string(what) + ": launch grid beyond 2^32 work-items");
}

// ---------------------------------------------------------------- worker pool
WorkerPool::~WorkerPool() {
    {
        std::lock_guard<std::mutex> lk(mu_);
        quit_ = true;
    }
    cv_work_.notify_all();
    for (auto &t : threads_) t.join();
}

void WorkerPool::loop(int k) {
    std::unique_lock<std::mutex> lk(mu_);
    while (true) {
        cv_work_.wait(lk, [&] { return quit_ || ready_[k]; });
        if (!ready_[k]) return;   // quit with nothing left to run
        const std::function<void(int)> *fn = job_[k];
        ready_[k] = 0;
        lk.unlock();
        (void)hipSetDevice(device_);   // jobs select the device again and report a failure
        (*fn)(k);
        lk.lock();
        if (--pending_ == 0) cv_done_.notify_all();
    }
}

void WorkerPool::run(int n, const std::function<void(int)> &fn) {
    if (n <= 0) return;
    std::unique_lock<std::mutex> lk(mu_);
    while ((int)threads_.size() < n) {
        const int k = (int)threads_.size();
        job_.push_back(nullptr);
        ready_.push_back(0);
        threads_.emplace_back([this, k] { loop(k); });
    }
    for (int k = 0; k < n; ++k) {
        job_[k] = &fn;
        ready_[k] = 1;
    }
    pending_ = n;
    cv_work_.notify_all();
    cv_done_.wait(lk, [&] { return pending_ == 0; });
}

}  // namespace pdmrg
