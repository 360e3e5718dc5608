// Environment update that allocates no device memory (env_update_noalloc):
// its intermediates and the device copies of its work lists live in a
// file-scope device array, one copy per GPU, held until the process ends.
#include "internal.hpp"

#include <mutex>

namespace pdmrg {

// 64 MiB per device: the two intermediates of the update plus its work lists.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};   // device address of `scratch` on each device

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }
}  // namespace

// Called by pdmrg_ctx_create with `device` current: resolves the device
// address of the array on that device (once per device).
void noalloc_init(int device) {
    PD_REQUIRE(device >= 0 && device < kMaxDevices, PDMRG_EINVAL, "noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return;
    void *p = nullptr;
    HIP_OK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    PD_REQUIRE(p != nullptr, PDMRG_EHIP, "noalloc: no device address for the scratch array");
    g_scratch[device] = p;
}

namespace {
void *scratch_of(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    PD_REQUIRE(device >= 0 && device < kMaxDevices && g_scratch[device], PDMRG_EINVAL,
               "env_update_noalloc: scratch not set up on this device (create the context first)");
    return g_scratch[device];
}

// Lays records out in the scratch array (256-byte aligned) and copies them in.
struct Packer {
    char *base;
    size_t used = 0;
    template <class T>
    size_t reserve(const std::vector<T> &v) {
        const size_t at = used;
        used = align256(used + std::max<size_t>(v.size() * sizeof(T), 1));
        return at;
    }
    template <class T>
    const T *put(const std::vector<T> &v, size_t at, hipStream_t s) {
        if (!v.empty()) HIP_OK(hipMemcpyAsync(base + at, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
        return reinterpret_cast<const T *>(base + at);
    }
};

struct ListAt {
    size_t items, segs, tiles, ftiles, rowoff;
};
ListAt reserve_list(Packer &pk, const GemmList &g) {
    ListAt a;
    a.items = pk.reserve(g.items);
    a.segs = pk.reserve(g.segs);
    a.tiles = pk.reserve(g.tiles);
    a.ftiles = pk.reserve(g.ftiles);
    a.rowoff = pk.reserve(g.rowoff);
    return a;
}
GemmDev put_list(Packer &pk, const GemmList &g, const ListAt &a, hipStream_t s) {
    return GemmDev{pk.put(g.items, a.items, s), pk.put(g.segs, a.segs, s), pk.put(g.tiles, a.tiles, s),
                   pk.put(g.ftiles, a.ftiles, s), pk.put(g.rowoff, a.rowoff, s)};
}
}  // namespace

}  // namespace pdmrg

using namespace pdmrg;

extern "C" int env_update_noalloc(pdmrg_ctx *ctx, int dir, const pdmrg_bond *bl, const pdmrg_bond *br,
                                  const pdmrg_phys *phys, const pdmrg_mpo_site *W, const double *env_in_dev,
                                  const double *site_dev, double *env_out_dev, int prec) {
    try {
        PD_REQUIRE(ctx && env_in_dev && site_dev && env_out_dev, PDMRG_EINVAL, "env_update_noalloc: null argument");
        PD_REQUIRE(dir == 1 || dir == -1, PDMRG_EINVAL, "env_update_noalloc: dir must be +1 or -1");
        PD_REQUIRE(prec == PDMRG_F64, PDMRG_EINVAL, "env_update_noalloc: only FP64 environments are supported");
        hipStream_t s = ctx->stream;
        EnvPlan plan;   // host work lists only: nothing is uploaded
        plan.build(dir, Bond::from(bl), Bond::from(br), Phys::from(phys), MpoSite::from(W), s, false);
        plan.g1.build_tiles();
        plan.w.build_tiles();
        plan.g3.build_tiles();
        Packer pk{static_cast<char *>(scratch_of(ctx->device))};
        const size_t u1 = pk.used;
        pk.used = align256(pk.used + (size_t)std::max<int64_t>(plan.nU1, 1) * sizeof(double));
        const size_t u2 = pk.used;
        pk.used = align256(pk.used + (size_t)std::max<int64_t>(plan.nU2, 1) * sizeof(double));
        const ListAt a1 = reserve_list(pk, plan.g1), a3 = reserve_list(pk, plan.g3);
        const size_t wt = pk.reserve(plan.w.tasks), ws = pk.reserve(plan.w.srcs), wl = pk.reserve(plan.w.tiles);
        PD_REQUIRE(pk.used <= kScratchBytes, PDMRG_EINVAL,
                   "env_update_noalloc: the update needs " + std::to_string(pk.used) +
                       " bytes of scratch, more than its limit of " + std::to_string(kScratchBytes) +
                       " (use env_update)");
        const GemmDev d1 = put_list(pk, plan.g1, a1, s), d3 = put_list(pk, plan.g3, a3, s);
        const LcDev dw{pk.put(plan.w.tasks, wt, s), pk.put(plan.w.srcs, ws, s), pk.put(plan.w.tiles, wl, s)};
        plan.run(GemmPrec::F64, env_in_dev, site_dev, env_out_dev, pk.base + u1, pk.base + u2, d1, dw, d3, s);
        // the host lists the copies read from live until here
        HIP_OK(hipStreamSynchronize(s));
    } catch (const Error &e) {
        set_last_error(e.what());
        return e.code;
    } catch (const std::exception &e) {
        set_last_error(e.what());
        return PDMRG_EINVAL;
    }
    return PDMRG_OK;
}
