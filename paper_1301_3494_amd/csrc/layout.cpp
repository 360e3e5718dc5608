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

// Caching device allocator behind DevBuf.  Sizes are rounded up to a power of
// two (at least 256 bytes); released blocks go to a pending list and become
// reusable only after one device-wide synchronisation, so a block can never be
// handed out while a kernel launched before its release still uses it.  That
// synchronisation waits for every stream (concurrent regions included), so it
// is taken only once the pending blocks hold kRecycleBytes; below that a miss
// allocates a new block.  Cached blocks are kept until the process ends.
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
struct DeviceCache {
    std::map<std::pair<int, size_t>, std::vector<void *>> free_, pending_;
    size_t pending_bytes = 0;
};
DeviceCache &cache() {
    static DeviceCache *c = new DeviceCache();   // never destroyed: no hipFree after runtime teardown
    return *c;
}
size_t size_class(size_t n) {
    size_t c = 256;
    while (c < n) c <<= 1;
    return c;
}
void recycle(DeviceCache &c) {
    HIP_OK(hipDeviceSynchronize());
    for (auto &kv : c.pending_) {
        auto &dst = c.free_[kv.first];
        dst.insert(dst.end(), kv.second.begin(), kv.second.end());
        kv.second.clear();
    }
    c.pending_bytes = 0;
}
}  // namespace

void DevBuf::alloc(size_t n) {
    if (n == 0) n = 16;
    int dev = 0;
    HIP_OK(hipGetDevice(&dev));
    const size_t cls = size_class(n);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    DeviceCache &c = cache();
    auto key = std::make_pair(dev, cls);
    auto it = c.free_.find(key);
    if ((it == c.free_.end() || it->second.empty()) && c.pending_bytes >= kRecycleBytes) {
        recycle(c);
        it = c.free_.find(key);
    }
    if (it != c.free_.end() && !it->second.empty()) {
        ptr = it->second.back();
        it->second.pop_back();
        bytes = cls;
        poison(ptr, cls);
        return;
    }
    hipError_t e = hipMalloc(&ptr, cls);
    if (e != hipSuccess) {
        // release every cached block and retry once
        (void)hipGetLastError();
        HIP_OK(hipDeviceSynchronize());
        for (auto *m : {&c.free_, &c.pending_})
            for (auto &kv : *m) {
                for (void *p : kv.second) (void)hipFree(p);
                kv.second.clear();
            }
        c.pending_bytes = 0;
        e = hipMalloc(&ptr, cls);
    }
    if (e != hipSuccess) {
        ptr = nullptr;
        bytes = 0;
        throw Error(PDMRG_ENOMEM, "hipMalloc of " + std::to_string(cls) + " bytes failed: " + hipGetErrorString(e));
    }
    bytes = cls;
    poison(ptr, cls);
}

void DevBuf::release() {
    if (ptr) {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_cache_mu);
            DeviceCache &c = cache();
            c.pending_[std::make_pair(dev, bytes)].push_back(ptr);
            c.pending_bytes += bytes;
        }
    }
    ptr = nullptr;
    bytes = 0;
}

}  // namespace pdmrg
